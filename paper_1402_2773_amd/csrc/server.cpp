// server.cpp -- continuous-batching decode runtime over resident slot pools.
//
// Every request is a run of frames of one code.  It is admitted when its
// code's pool has a free contiguous slot range (the pools are allocated once,
// so admission is by free HBM), filled by the client, committed, and then
// joined with every other committed request of its code into one segmented
// launch (ngdbf_decode_segments) on the next library stream.  Launches of
// different codes and of successive pumps run concurrently; completion is
// observed with events, never by waiting on the device.  Because each
// request keeps its own noise key (seed, frame index), its results do not
// depend on what it was launched with.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <deque>
#include <map>
#include <mutex>
#include <unordered_map>
#include <vector>

#include "../../include/ngdbf.h"

namespace ngdbf_host {
int set_error(int code, const char *msg);  // decode.hip: the per-thread message
}

namespace {

// Failures are reported through ngdbf_last_error, like every other call.
ngdbf_status sfail(int code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
ngdbf_status sfail(int code, const char *fmt, ...) {
  char msg[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(msg, sizeof msg, fmt, ap);
  va_end(ap);
  return (ngdbf_status)ngdbf_host::set_error(code, msg);
}

// First-fit allocator of contiguous slot ranges, coalescing on release.
class SlotAllocator {
 public:
  explicit SlotAllocator(int64_t capacity) { free_[0] = capacity; }
  bool take(int64_t count, int64_t *first) {
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= count) {
        *first = it->first;
        const int64_t rest_start = it->first + count, rest_len = it->second - count;
        free_.erase(it);
        if (rest_len) free_[rest_start] = rest_len;
        return true;
      }
    }
    return false;
  }
  void give(int64_t first, int64_t count) {
    auto next = free_.lower_bound(first);
    if (next != free_.end() && first + count == next->first) {
      count += next->second;
      next = free_.erase(next);
    }
    if (next != free_.begin()) {
      auto prev = std::prev(next);
      if (prev->first + prev->second == first) {
        prev->second += count;
        return;
      }
    }
    free_[first] = count;
  }

 private:
  std::map<int64_t, int64_t> free_;  // start -> length
};

enum class State { kAdmitted, kCommitted, kLaunched, kDone };

struct Request {
  int code;
  int64_t first, count;
  uint64_t seed, frame_base;
  State state;
  hipEvent_t ready;  // recorded at commit on the client's stream
};

struct CodePool {
  ngdbf_code *code;
  ngdbf_params params;
  int64_t capacity;
  int32_t n, nbytes;
  float *y = nullptr, *sigma = nullptr;
  uint8_t *bits = nullptr, *conv = nullptr;
  int32_t *iters = nullptr;
  SlotAllocator alloc{0};
  std::deque<uint64_t> ready;  // committed, not yet launched (FIFO)
};

// Host/device staging for one launch's segment table; reused once the
// launch has finished.
struct LaunchSlot {
  ngdbf_segment *host = nullptr;  // pinned
  ngdbf_segment *dev = nullptr;
  hipEvent_t done = nullptr;
  bool busy = false;
  int stream = -1;  // library stream of the launch in flight
  std::vector<uint64_t> tickets;
};

constexpr int kMaxSegments = 32768;  // requests per launch
constexpr int kLaunchSlots = 32;     // launches in flight

}  // namespace

struct ngdbf_server {
  int device = 0;
  std::mutex mu;
  std::vector<CodePool> pools;
  std::vector<hipStream_t> streams;
  std::vector<int> stream_load;  // launches in flight per stream
  std::vector<LaunchSlot> launches;
  std::deque<int> inflight;  // launch slot indices, in launch order
  std::unordered_map<uint64_t, Request> requests;
  std::unordered_map<hipEvent_t, int> ready_refs;  // commit event -> requests not yet launched
  uint64_t next_ticket = 1;
  int max_per_launch = kMaxSegments;
  int per_stream = 1;
};

namespace {

void destroy_server(ngdbf_server *s) {
  for (auto &l : s->launches) {
    if (l.done) (void)hipEventSynchronize(l.done);
  }
  for (auto &l : s->launches) {
    if (l.host) (void)hipHostFree(l.host);
    if (l.dev) (void)hipFree(l.dev);
    if (l.done) (void)hipEventDestroy(l.done);
  }
  for (auto &kv : s->ready_refs) (void)hipEventDestroy(kv.first);
  for (auto st : s->streams) (void)hipStreamDestroy(st);
  for (auto &p : s->pools) {
    (void)hipFree(p.y);
    (void)hipFree(p.sigma);
    (void)hipFree(p.bits);
    (void)hipFree(p.iters);
    (void)hipFree(p.conv);
  }
  delete s;
}

}  // namespace

extern "C" {

ngdbf_status ngdbf_server_create(int32_t n_codes, ngdbf_code *const *codes, const ngdbf_params *params,
                        const int64_t *pool_frames, int32_t n_streams,
                        int32_t max_requests_per_launch, int32_t launches_per_stream,
                        ngdbf_server **out) {
  if (!out) return sfail(NGDBF_EINVAL, "out is NULL");
  *out = nullptr;
  if (n_codes < 1 || !codes || !params || !pool_frames)
    return sfail(NGDBF_EINVAL, "codes, params and pool sizes are required");
  if (n_streams < 1 || n_streams > 16) return sfail(NGDBF_EINVAL, "n_streams must be in [1, 16]");
  if (max_requests_per_launch < 1 || max_requests_per_launch > kMaxSegments)
    return sfail(NGDBF_EINVAL, "max_requests_per_launch must be in [1, %d]", kMaxSegments);
  if (launches_per_stream < 1 || (int64_t)launches_per_stream * n_streams > kLaunchSlots)
    return sfail(NGDBF_EINVAL, "launches_per_stream must be >= 1 with n_streams * launches_per_stream <= %d",
                 kLaunchSlots);
  ngdbf_server *s = new ngdbf_server();
  s->max_per_launch = max_requests_per_launch;
  s->per_stream = launches_per_stream;
  if (hipGetDevice(&s->device) != hipSuccess) {
    delete s;
    return sfail(NGDBF_EDEVICE, "no HIP device");
  }
  s->pools.resize((size_t)n_codes);
  for (int i = 0; i < n_codes; ++i) {
    CodePool &p = s->pools[(size_t)i];
    int32_t n = 0, m = 0, nnz = 0;
    if (!codes[i] || ngdbf_code_info(codes[i], &n, &m, &nnz) != NGDBF_OK) {
      destroy_server(s);
      return sfail(NGDBF_EINVAL, "code %d is invalid", i);
    }
    if (pool_frames[i] < 1 || params[i].y_format != NGDBF_Y_F32) {
      destroy_server(s);
      return sfail(NGDBF_EINVAL, "code %d: pool size >= 1 and float32 samples are required", i);
    }
    p.code = codes[i];
    p.params = params[i];
    p.capacity = pool_frames[i];
    p.n = n;
    p.nbytes = (n + 7) / 8;
    p.alloc = SlotAllocator(p.capacity);
    const size_t F = (size_t)p.capacity;
    if (hipMalloc((void **)&p.y, F * (size_t)n * 4) != hipSuccess ||
        hipMalloc((void **)&p.sigma, F * 4) != hipSuccess ||
        hipMalloc((void **)&p.bits, F * (size_t)p.nbytes) != hipSuccess ||
        hipMalloc((void **)&p.iters, F * 4) != hipSuccess ||
        hipMalloc((void **)&p.conv, F) != hipSuccess) {
      destroy_server(s);
      return sfail(NGDBF_ENOMEM, "pool of %lld frames for code %d does not fit",
                   (long long)p.capacity, i);
    }
  }
  for (int i = 0; i < n_streams; ++i) {
    hipStream_t st = nullptr;
    // default priority, non-blocking with respect to the null stream
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
      destroy_server(s);
      return sfail(NGDBF_EDEVICE, "stream creation failed");
    }
    s->streams.push_back(st);
    s->stream_load.push_back(0);
  }
  s->launches.resize(kLaunchSlots);
  for (auto &l : s->launches) {
    if (hipHostMalloc((void **)&l.host, sizeof(ngdbf_segment) * kMaxSegments, 0) != hipSuccess ||
        hipMalloc((void **)&l.dev, sizeof(ngdbf_segment) * kMaxSegments) != hipSuccess ||
        hipEventCreateWithFlags(&l.done, hipEventDisableTiming) != hipSuccess) {
      destroy_server(s);
      return sfail(NGDBF_ENOMEM, "launch staging allocation failed");
    }
  }
  *out = s;
  return NGDBF_OK;
}

ngdbf_status ngdbf_server_destroy(ngdbf_server *server) {
  if (server) destroy_server(server);
  return NGDBF_OK;
}

ngdbf_status ngdbf_server_pools(ngdbf_server *s, int32_t code_index, float **y, float **sigma,
                       uint8_t **bits, int32_t **iters, uint8_t **converged) {
  if (!s || code_index < 0 || code_index >= (int)s->pools.size())
    return sfail(NGDBF_EINVAL, "bad server or code index");
  const CodePool &p = s->pools[(size_t)code_index];
  if (y) *y = p.y;
  if (sigma) *sigma = p.sigma;
  if (bits) *bits = p.bits;
  if (iters) *iters = p.iters;
  if (converged) *converged = p.conv;
  return NGDBF_OK;
}

ngdbf_status ngdbf_server_admit(ngdbf_server *s, int32_t n_requests, const int32_t *code_index,
                       const int64_t *n_frames, const uint64_t *seed, const uint64_t *frame_base,
                       uint64_t *tickets, int64_t *first_slots, int32_t *n_admitted) {
  if (!s || n_requests < 0 || !n_admitted) return sfail(NGDBF_EINVAL, "bad arguments");
  *n_admitted = 0;
  if (n_requests == 0) return NGDBF_OK;
  if (!code_index || !n_frames || !seed || !frame_base || !tickets || !first_slots)
    return sfail(NGDBF_EINVAL, "request arrays are required");
  std::lock_guard<std::mutex> g(s->mu);
  for (int r = 0; r < n_requests; ++r) {
    const int c = code_index[r];
    if (c < 0 || c >= (int)s->pools.size()) return sfail(NGDBF_EINVAL, "request %d: bad code", r);
    CodePool &p = s->pools[(size_t)c];
    if (n_frames[r] < 1 || n_frames[r] > p.capacity)
      return sfail(NGDBF_EINVAL, "request %d: %lld frames for a pool of %lld", r,
                   (long long)n_frames[r], (long long)p.capacity);
    int64_t first = 0;
    if (!p.alloc.take(n_frames[r], &first)) break;  // no room: stop here, in order
    const uint64_t t = s->next_ticket++;
    s->requests[t] = Request{c, first, n_frames[r], seed[r], frame_base[r], State::kAdmitted, nullptr};
    tickets[r] = t;
    first_slots[r] = first;
    *n_admitted = r + 1;
  }
  return NGDBF_OK;
}

ngdbf_status ngdbf_server_commit(ngdbf_server *s, int32_t n, const uint64_t *tickets, void *stream) {
  if (!s || n < 0 || (n > 0 && !tickets)) return sfail(NGDBF_EINVAL, "bad arguments");
  if (n == 0) return NGDBF_OK;
  std::lock_guard<std::mutex> g(s->mu);
  for (int i = 0; i < n; ++i) {
    auto it = s->requests.find(tickets[i]);
    if (it == s->requests.end() || it->second.state != State::kAdmitted)
      return sfail(NGDBF_EINVAL, "ticket %llu is not an admitted request",
                   (unsigned long long)tickets[i]);
  }
  hipEvent_t ev = nullptr;
  if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess ||
      hipEventRecord(ev, (hipStream_t)stream) != hipSuccess)
    return sfail(NGDBF_EDEVICE, "commit event failed");
  for (int i = 0; i < n; ++i) {
    Request &r = s->requests[tickets[i]];
    r.state = State::kCommitted;
    r.ready = ev;
    s->pools[(size_t)r.code].ready.push_back(tickets[i]);
  }
  s->ready_refs[ev] = n;  // destroyed once the last of these requests is launched
  return NGDBF_OK;
}

ngdbf_status ngdbf_server_pump(ngdbf_server *s, int32_t *n_launched) {
  if (!s) return sfail(NGDBF_EINVAL, "server is NULL");
  std::lock_guard<std::mutex> g(s->mu);
  int launched = 0;
  for (;;) {
    // the code whose oldest committed request was admitted first (tickets grow)
    int c = -1;
    for (int i = 0; i < (int)s->pools.size(); ++i) {
      const CodePool &q = s->pools[(size_t)i];
      if (!q.ready.empty() && (c < 0 || q.ready.front() < s->pools[(size_t)c].ready.front())) c = i;
    }
    if (c < 0) break;
    // the least loaded stream with room; none: the requests wait, and grow the
    // next launch
    int si = -1;
    for (int i = 0; i < (int)s->streams.size(); ++i)
      if (s->stream_load[(size_t)i] < s->per_stream &&
          (si < 0 || s->stream_load[(size_t)i] < s->stream_load[(size_t)si]))
        si = i;
    if (si < 0) break;
    int slot = -1;
    for (int l = 0; l < (int)s->launches.size(); ++l)
      if (!s->launches[(size_t)l].busy) {
        slot = l;
        break;
      }
    if (slot < 0) break;
    CodePool &p = s->pools[(size_t)c];
    LaunchSlot &L = s->launches[(size_t)slot];
    L.tickets.clear();
    hipStream_t st = s->streams[(size_t)si];
    std::vector<hipEvent_t> waits;
    int64_t frames = 0;
    int nseg = 0;
    while (!p.ready.empty() && nseg < s->max_per_launch) {
      const uint64_t t = p.ready.front();
      p.ready.pop_front();
      Request &r = s->requests[t];
      L.host[nseg] = ngdbf_segment{r.first, frames, r.seed, r.frame_base};
      frames += r.count;
      ++nseg;
      L.tickets.push_back(t);
      r.state = State::kLaunched;
      if (std::find(waits.begin(), waits.end(), r.ready) == waits.end()) waits.push_back(r.ready);
    }
    for (hipEvent_t e : waits) {
      if (hipStreamWaitEvent(st, e, 0) != hipSuccess) return sfail(NGDBF_EDEVICE, "wait failed");
    }
    if (hipMemcpyAsync(L.dev, L.host, sizeof(ngdbf_segment) * (size_t)nseg,
                       hipMemcpyHostToDevice, st) != hipSuccess)
      return sfail(NGDBF_EDEVICE, "segment upload failed");
    const int rc = ngdbf_decode_segments(p.code, p.y, p.sigma, 0.0f, p.capacity, &p.params, L.dev,
                                         nseg, frames, p.bits, p.iters, p.conv, st);
    if (rc) return sfail(rc, "launch failed: %s", ngdbf_last_error());
    if (hipEventRecord(L.done, st) != hipSuccess) return sfail(NGDBF_EDEVICE, "record failed");
    L.busy = true;
    L.stream = si;
    ++s->stream_load[(size_t)si];
    s->inflight.push_back(slot);
    ++launched;
    // the waits are queued: drop this launch's references to commit events
    for (uint64_t t : L.tickets) {
      Request &r = s->requests[t];
      auto ref = s->ready_refs.find(r.ready);
      if (ref != s->ready_refs.end() && --ref->second == 0) {
        (void)hipEventDestroy(ref->first);  // released once its record has completed
        s->ready_refs.erase(ref);
      }
      r.ready = nullptr;
    }
  }
  if (n_launched) *n_launched = launched;
  return NGDBF_OK;
}

ngdbf_status ngdbf_server_poll(ngdbf_server *s, int32_t capacity, uint64_t *tickets, int32_t *n_done) {
  if (!s || capacity < 0 || !n_done || (capacity > 0 && !tickets))
    return sfail(NGDBF_EINVAL, "bad arguments");
  *n_done = 0;
  std::lock_guard<std::mutex> g(s->mu);
  for (auto it = s->inflight.begin(); it != s->inflight.end();) {
    LaunchSlot &L = s->launches[(size_t)*it];
    if ((int64_t)*n_done + (int64_t)L.tickets.size() > capacity) break;
    const hipError_t q = hipEventQuery(L.done);
    if (q == hipErrorNotReady) {
      ++it;
      continue;
    }
    if (q != hipSuccess) return sfail(NGDBF_EDEVICE, "launch failed: %s", hipGetErrorString(q));
    for (uint64_t t : L.tickets) {
      s->requests[t].state = State::kDone;
      tickets[(*n_done)++] = t;
    }
    L.tickets.clear();
    L.busy = false;
    --s->stream_load[(size_t)L.stream];
    L.stream = -1;
    it = s->inflight.erase(it);
  }
  return NGDBF_OK;
}

ngdbf_status ngdbf_server_release(ngdbf_server *s, int32_t n, const uint64_t *tickets) {
  if (!s || n < 0 || (n > 0 && !tickets)) return sfail(NGDBF_EINVAL, "bad arguments");
  std::lock_guard<std::mutex> g(s->mu);
  for (int i = 0; i < n; ++i) {
    auto it = s->requests.find(tickets[i]);
    if (it == s->requests.end() || it->second.state != State::kDone)
      return sfail(NGDBF_EINVAL, "ticket %llu is not a finished request",
                   (unsigned long long)tickets[i]);
    s->pools[(size_t)it->second.code].alloc.give(it->second.first, it->second.count);
    s->requests.erase(it);
  }
  return NGDBF_OK;
}

}  // extern "C"
