// server.hip -- continuous-batching query server over compressed streams
// (host code; the declarations and semantics are in include/hoszp.h).
//
// A server is a set of execution slots plus one device memory pool.  Queries
// wait in a host queue until a slot is free and the pool can hold what the
// query needs (its output stream and, on the decompress-then-compute path, its
// float32 intermediates); then they are launched on the slot's own stream with
// the slot's own context, so queries admitted at different times overlap on
// the device.  Completion is detected without blocking (an event per slot and
// a pinned copy of the slot's result records).  Single-threaded: one host
// thread drives a server.

#include <math.h>

#include <chrono>
#include <deque>
#include <map>
#include <new>
#include <unordered_map>
#include <vector>

#include "hoszp_internal.h"

namespace {

constexpr uint64_t kAlign = 256;
constexpr int kRecords = 4;  // result records per slot
constexpr uint64_t kNoIndex = ~uint64_t(0);

uint64_t up(uint64_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// First-fit allocator over one device arena, with coalescing of free ranges.
class Pool {
 public:
  bool init(uint64_t bytes) {
    size_ = up(bytes);
    if (hipMalloc(&base_, size_) != hipSuccess) {
      base_ = nullptr;
      return false;
    }
    free_[0] = size_;
    return true;
  }
  void release_all() {
    if (base_) (void)hipFree(base_);
    base_ = nullptr;
  }
  uint8_t* alloc(uint64_t bytes) {
    bytes = up(bytes ? bytes : 1);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < bytes) continue;
      const uint64_t off = it->first, len = it->second;
      free_.erase(it);
      if (len > bytes) free_[off + bytes] = len - bytes;
      used_[off] = bytes;
      in_use_ += bytes;
      if (in_use_ > peak_) peak_ = in_use_;
      return static_cast<uint8_t*>(base_) + off;
    }
    return nullptr;
  }
  bool free(void* p) {
    if (!p) return true;
    const uint64_t off = uint64_t(static_cast<uint8_t*>(p) - static_cast<uint8_t*>(base_));
    auto u = used_.find(off);
    if (u == used_.end()) return false;
    uint64_t start = off, len = u->second;
    used_.erase(u);
    in_use_ -= len;
    auto next = free_.lower_bound(start);
    if (next != free_.end() && next->first == start + len) {
      len += next->second;
      free_.erase(next);
    }
    auto prev = free_.lower_bound(start);
    if (prev != free_.begin()) {
      --prev;
      if (prev->first + prev->second == start) {
        start = prev->first;
        len += prev->second;
        free_.erase(prev);
      }
    }
    free_[start] = len;
    return true;
  }
  uint64_t size() const { return size_; }
  uint64_t peak() const { return peak_; }

 private:
  void* base_ = nullptr;
  uint64_t size_ = 0, in_use_ = 0, peak_ = 0;
  std::map<uint64_t, uint64_t> free_;           // offset -> length
  std::unordered_map<uint64_t, uint64_t> used_;  // offset -> length
};

struct Pending {
  hoszp_request req;
  double submit_s;
  uint64_t index;  // replay index, or kNoIndex
};

struct Slot {
  hoszp_ctx* ctx = nullptr;
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  hoszp_result* d_res = nullptr;  // kRecords records
  hoszp_result* h_res = nullptr;  // pinned mirror
  bool busy = false;
  int records = 0;                // records the running query uses
  Pending job{};
  double admit_s = 0;
  uint8_t* out = nullptr;         // output stream (pool)
  uint8_t* tmp = nullptr;         // float32 intermediates (pool)
};

double clock_s(std::chrono::steady_clock::time_point t0) {
  return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

bool op_ok(uint32_t op) { return op <= HOSZP_OP_MUL; }

// Output stream bytes and float32 intermediate bytes of a query.
void needs(const hoszp_request& r, uint64_t& out, uint64_t& tmp) {
  const bool makes_stream = r.op == HOSZP_OP_NEGATE || r.op == HOSZP_OP_ADD || r.op == HOSZP_OP_MUL;
  out = 0;
  tmp = 0;
  if (r.path == HOSZP_PATH_HOMOMORPHIC) {
    if (r.op == HOSZP_OP_NEGATE) out = r.a_bytes;
    else if (makes_stream) out = hz::bound_bytes(r.n, r.block);
  } else {
    if (makes_stream) out = hz::bound_bytes(r.n, r.block);
    tmp = up(4 * r.n) * (r.op == HOSZP_OP_ADD ? 2 : 1);
  }
}

}  // namespace

struct hoszp_server {
  int device = 0;
  hoszp_server_config cfg{};
  std::chrono::steady_clock::time_point t0;
  Pool pool;
  std::vector<Slot> slots;
  void* d_records = nullptr;
  std::deque<Pending> queue;
  std::deque<hoszp_completion> done;         // finished, not yet returned by poll
  std::vector<std::pair<uint64_t, hoszp_completion>> replay_done;
  hoszp_server_stats st{};
};

namespace {

class DevScope {
 public:
  explicit DevScope(int dev) {
    ok_ = hipGetDevice(&prev_) == hipSuccess;
    if (ok_ && prev_ != dev) ok_ = hipSetDevice(dev) == hipSuccess, switched_ = ok_;
  }
  ~DevScope() {
    if (switched_) (void)hipSetDevice(prev_);
  }
  bool ok() const { return ok_; }

 private:
  int prev_ = 0;
  bool ok_ = false, switched_ = false;
};

// Enqueue a query's kernels on its slot; returns a host-detected error code.
int launch_query(Slot& sl, const hoszp_request& r) {
  hoszp_ctx* c = sl.ctx;
  void* st = sl.stream;
  hoszp_result* R = sl.d_res;
  const uint64_t cap = hz::bound_bytes(r.n, r.block);
  int rc = HOSZP_OK;
  sl.records = 1;
  if (r.path == HOSZP_PATH_HOMOMORPHIC) {
    switch (r.op) {
      case HOSZP_OP_MEAN: rc = hoszp_mean_async(c, r.d_a, r.a_bytes, R, st); break;
      case HOSZP_OP_VARIANCE: rc = hoszp_variance_async(c, r.d_a, r.a_bytes, R, st); break;
      case HOSZP_OP_NEGATE:
        rc = hoszp_negate_async(c, r.d_a, r.a_bytes, sl.out, r.a_bytes, R, st);
        break;
      case HOSZP_OP_ADD:
        rc = hoszp_add_async(c, r.d_a, r.a_bytes, r.d_b, r.b_bytes, sl.out, cap, R, st);
        break;
      default: rc = hoszp_mul_async(c, r.d_a, r.a_bytes, r.scalar, sl.out, cap, R, st); break;
    }
    return rc;
  }
  // decompress, float32 op in HBM, re-compress (or reduce)
  float* x = reinterpret_cast<float*>(sl.tmp);
  float* y = reinterpret_cast<float*>(sl.tmp + up(4 * r.n));
  sl.records = r.op == HOSZP_OP_ADD ? 3 : 2;
  rc = hoszp_decompress_async(c, r.d_a, r.a_bytes, x, r.n, R + 1, st);
  if (rc == HOSZP_OK && r.op == HOSZP_OP_ADD)
    rc = hoszp_decompress_async(c, r.d_b, r.b_bytes, y, r.n, R + 2, st);
  if (rc != HOSZP_OK) return rc;
  switch (r.op) {
    case HOSZP_OP_MEAN: return hoszp_f32_mean_async(c, x, r.n, R, st);
    case HOSZP_OP_VARIANCE: return hoszp_f32_variance_async(c, x, r.n, R, st);
    case HOSZP_OP_NEGATE: rc = hoszp_f32_negate_async(c, x, x, r.n, st); break;
    case HOSZP_OP_ADD: rc = hoszp_f32_add_async(c, x, y, x, r.n, st); break;
    default: rc = hoszp_f32_mul_async(c, x, r.scalar, x, r.n, st); break;
  }
  if (rc != HOSZP_OK) return rc;
  return hoszp_compress_async(c, x, r.n, r.eb, r.block, sl.out, cap, R, st);
}

void finish(hoszp_server* s, Slot& sl, int code, const hoszp_result* rec) {
  hoszp_completion cpl{};
  cpl.tag = sl.job.req.tag;
  cpl.op = sl.job.req.op;
  cpl.code = code;
  if (code == HOSZP_OK && rec) {
    // the first failing record decides the code (decompress before the op)
    for (int k = sl.records - 1; k >= 1 && cpl.code == HOSZP_OK; --k)
      if (rec[k].status) cpl.code = hoszp_status_code(rec[k].status);
    if (cpl.code == HOSZP_OK && rec[0].status) cpl.code = hoszp_status_code(rec[0].status);
    cpl.value = rec[0].value;
    cpl.out_bytes = rec[0].out_bytes;
  }
  cpl.submit_s = sl.job.submit_s;
  cpl.admit_s = sl.admit_s;
  cpl.done_s = clock_s(s->t0);
  s->pool.free(sl.tmp);
  sl.tmp = nullptr;
  if (sl.out && (cpl.code != HOSZP_OK || !s->cfg.keep_outputs)) {
    s->pool.free(sl.out);
    sl.out = nullptr;
  }
  cpl.d_out = sl.out;
  if (!cpl.d_out) cpl.out_bytes = cpl.code == HOSZP_OK ? cpl.out_bytes : 0;
  sl.out = nullptr;
  sl.busy = false;
  ++s->st.completed;
  if (cpl.code != HOSZP_OK) ++s->st.failed;
  if (sl.job.index != kNoIndex)
    s->replay_done.emplace_back(sl.job.index, cpl);
  else
    s->done.push_back(cpl);
}

// Try to start `p` on slot `sl`: false when the pool cannot hold it now.
bool admit(hoszp_server* s, Slot& sl, const Pending& p) {
  uint64_t out_b, tmp_b;
  needs(p.req, out_b, tmp_b);
  uint8_t* out = out_b ? s->pool.alloc(out_b) : nullptr;
  if (out_b && !out) return false;
  uint8_t* tmp = tmp_b ? s->pool.alloc(tmp_b) : nullptr;
  if (tmp_b && !tmp) {
    s->pool.free(out);
    return false;
  }
  sl.job = p;
  sl.out = out;
  sl.tmp = tmp;
  sl.busy = true;
  sl.admit_s = clock_s(s->t0);
  ++s->st.admitted;
  const int rc = launch_query(sl, p.req);
  if (rc != HOSZP_OK) {
    finish(s, sl, rc, nullptr);
    return true;
  }
  if (hipMemcpyAsync(sl.h_res, sl.d_res, sizeof(hoszp_result) * kRecords, hipMemcpyDeviceToHost,
                     sl.stream) != hipSuccess ||
      hipEventRecord(sl.done, sl.stream) != hipSuccess) {
    (void)hipStreamSynchronize(sl.stream);
    finish(s, sl, HOSZP_ERR_DEVICE, nullptr);
  }
  return true;
}

int check_request(const hoszp_server* s, const hoszp_request& r) {
  if (!op_ok(r.op) || r.path > HOSZP_PATH_TRADITIONAL || !r.d_a || r.reserved) return HOSZP_ERR_ARG;
  if (r.op == HOSZP_OP_ADD && !r.d_b) return HOSZP_ERR_ARG;
  if (r.n == 0 || r.n > hz::kMaxN || !hz::block_ok(r.block)) return HOSZP_ERR_ARG;
  if (r.path == HOSZP_PATH_TRADITIONAL && !(r.eb > 0.0 && isfinite(r.eb))) return HOSZP_ERR_ARG;
  if (r.op == HOSZP_OP_MUL && !isfinite(r.scalar)) return HOSZP_ERR_ARG;
  uint64_t out_b, tmp_b;
  needs(r, out_b, tmp_b);
  if (up(out_b) + up(tmp_b) > s->pool.size()) return HOSZP_ERR_CAPACITY;
  return HOSZP_OK;
}

void enqueue(hoszp_server* s, const hoszp_request& r, uint64_t index) {
  s->queue.push_back(Pending{r, clock_s(s->t0), index});
  ++s->st.submitted;
  if (s->queue.size() > s->st.queue_peak) s->st.queue_peak = s->queue.size();
}

// Collect finished slots, then admit queued queries into free slots.
int progress(hoszp_server* s) {
  for (Slot& sl : s->slots) {
    if (!sl.busy) continue;
    const hipError_t e = hipEventQuery(sl.done);
    if (e == hipErrorNotReady) continue;
    if (e != hipSuccess) {
      (void)hipGetLastError();
      finish(s, sl, HOSZP_ERR_DEVICE, nullptr);
      continue;
    }
    finish(s, sl, HOSZP_OK, sl.h_res);
  }
  if (s->queue.empty()) return HOSZP_OK;
  const double now = clock_s(s->t0);
  for (Slot& sl : s->slots) {
    if (sl.busy) continue;
    bool started = false;
    size_t scanned = 0;
    for (auto it = s->queue.begin(); it != s->queue.end() && scanned < 64; ++it, ++scanned) {
      if (admit(s, sl, *it)) {
        s->queue.erase(it);
        started = true;
        break;
      }
      // the oldest query may be passed only while it is young
      if (it == s->queue.begin() && now - it->submit_s > s->cfg.starve_s) break;
    }
    if (!started || s->queue.empty()) break;
  }
  return HOSZP_OK;
}

}  // namespace

extern "C" {

int hoszp_server_create(int device, const hoszp_server_config* cfg, hoszp_server** out) {
  if (!out) return HOSZP_ERR_ARG;
  *out = nullptr;
  if (!cfg || cfg->slots < 1 || cfg->slots > 64 || cfg->pool_bytes == 0 || cfg->keep_outputs > 1 ||
      !(cfg->starve_s >= 0.0))
    return HOSZP_ERR_ARG;
  DevScope scope(device);
  if (!scope.ok()) return HOSZP_ERR_DEVICE;
  hoszp_server* s = new (std::nothrow) hoszp_server();
  if (!s) return HOSZP_ERR_NOMEM;
  s->device = device;
  s->cfg = *cfg;
  if (s->cfg.starve_s == 0.0) s->cfg.starve_s = 0.05;
  s->t0 = std::chrono::steady_clock::now();
  int rc = s->pool.init(cfg->pool_bytes) ? HOSZP_OK : HOSZP_ERR_NOMEM;
  const size_t rec_b = sizeof(hoszp_result) * kRecords;
  if (rc == HOSZP_OK && hipMalloc(&s->d_records, rec_b * cfg->slots) != hipSuccess)
    rc = HOSZP_ERR_NOMEM;
  s->slots.resize(cfg->slots);
  for (uint32_t k = 0; k < cfg->slots && rc == HOSZP_OK; ++k) {
    Slot& sl = s->slots[k];
    rc = hoszp_ctx_create(device, &sl.ctx);
    if (rc != HOSZP_OK) break;
    if (hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) != hipSuccess) {
      rc = HOSZP_ERR_DEVICE;
      break;
    }
    if (hipHostMalloc(reinterpret_cast<void**>(&sl.h_res), rec_b, hipHostMallocDefault) !=
        hipSuccess) {
      sl.h_res = nullptr;
      rc = HOSZP_ERR_NOMEM;
      break;
    }
    sl.d_res = reinterpret_cast<hoszp_result*>(static_cast<uint8_t*>(s->d_records) + k * rec_b);
  }
  if (rc == HOSZP_OK && (hipMemset(s->d_records, 0, rec_b * cfg->slots) != hipSuccess ||
                         hipDeviceSynchronize() != hipSuccess))
    rc = HOSZP_ERR_DEVICE;
  s->st.pool_bytes = s->pool.size();
  if (rc != HOSZP_OK) {
    hoszp_server_destroy(s);
    return rc;
  }
  *out = s;
  return HOSZP_OK;
}

int hoszp_server_submit(hoszp_server* s, const hoszp_request* req) {
  if (!s || !req) return HOSZP_ERR_ARG;
  const int rc = check_request(s, *req);
  if (rc != HOSZP_OK) return rc;
  enqueue(s, *req, kNoIndex);
  return HOSZP_OK;
}

int hoszp_server_poll(hoszp_server* s, hoszp_completion* out, uint32_t max_out, uint32_t* n_out) {
  if (!s || !n_out || (max_out && !out)) return HOSZP_ERR_ARG;
  DevScope scope(s->device);
  if (!scope.ok()) return HOSZP_ERR_DEVICE;
  progress(s);
  uint32_t n = 0;
  while (n < max_out && !s->done.empty()) {
    out[n++] = s->done.front();
    s->done.pop_front();
  }
  *n_out = n;
  return HOSZP_OK;
}

uint64_t hoszp_server_pending(const hoszp_server* s) {
  if (!s) return 0;
  uint64_t busy = 0;
  for (const Slot& sl : s->slots) busy += sl.busy;
  return busy + s->queue.size();
}

int hoszp_server_release(hoszp_server* s, void* d_out) {
  if (!s || !d_out) return HOSZP_ERR_ARG;
  return s->pool.free(d_out) ? HOSZP_OK : HOSZP_ERR_ARG;
}

int hoszp_server_replay(hoszp_server* s, const hoszp_request* reqs, const double* arrival_s,
                        uint64_t count, hoszp_completion* out, double* start_s) {
  if (!s || (count && (!reqs || !arrival_s || !out))) return HOSZP_ERR_ARG;
  for (uint64_t i = 0; i < count; ++i) {
    const int rc = check_request(s, reqs[i]);
    if (rc != HOSZP_OK) return rc;
    if (!(arrival_s[i] >= 0.0) || (i && arrival_s[i] < arrival_s[i - 1])) return HOSZP_ERR_ARG;
  }
  DevScope scope(s->device);
  if (!scope.ok()) return HOSZP_ERR_DEVICE;
  s->replay_done.clear();
  s->replay_done.reserve(count);
  const double start = clock_s(s->t0);
  if (start_s) *start_s = start;
  uint64_t next = 0, finished = 0;
  while (finished < count) {
    const double t = clock_s(s->t0) - start;
    while (next < count && arrival_s[next] <= t) enqueue(s, reqs[next], next), ++next;
    progress(s);
    for (auto& d : s->replay_done) out[d.first] = d.second;
    finished += s->replay_done.size();
    s->replay_done.clear();
  }
  return HOSZP_OK;
}

int hoszp_server_stats_get(const hoszp_server* s, hoszp_server_stats* out) {
  if (!s || !out) return HOSZP_ERR_ARG;
  *out = s->st;
  out->pool_peak = s->pool.peak();
  return HOSZP_OK;
}

int hoszp_server_destroy(hoszp_server* s) {
  if (!s) return HOSZP_OK;
  DevScope scope(s->device);
  for (Slot& sl : s->slots) {
    if (sl.stream) (void)hipStreamSynchronize(sl.stream);
    if (sl.done) (void)hipEventDestroy(sl.done);
    if (sl.stream) (void)hipStreamDestroy(sl.stream);
    if (sl.h_res) (void)hipHostFree(sl.h_res);
    if (sl.ctx) (void)hoszp_ctx_destroy(sl.ctx);
  }
  if (s->d_records) (void)hipFree(s->d_records);
  s->pool.release_all();
  delete s;
  return HOSZP_OK;
}

}  // extern "C"
