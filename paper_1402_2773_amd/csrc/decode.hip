// decode.hip -- host side of the decoder: code handles, launch shapes,
// validation, the multi-bit binary32 kernels' instantiations, the noise
// probes and the C ABI of ngdbf.h.  The kernel itself is in kernel.h; the
// extended decoders (single-bit, mode switching, quantized, noise reuse) are
// instantiated in decode_ext.hip, one object per family.

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <cmath>
#include <cstdarg>

#include <algorithm>
#include <atomic>
#include <mutex>
#include <vector>

#include "../../include/ngdbf.h"
#include "noise.h"

#include "host.h"
#include "kernel.h"

namespace ngdbf {

// ---------------------------------------------------------------- probes

// zero n bytes (the trace rows; a kernel rather than a memset node, so that
// a captured graph clears them on every replay)
__global__ void clear_bytes_kernel(uint8_t *p, size_t n) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = 0;
}

__global__ void probe_radius_kernel(uint32_t start, uint32_t count, float *out) {
  const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < count) out[j] = bm_radius(start + j);
}

__global__ void probe_turn_kernel(uint32_t start, uint32_t count, float *co, float *si) {
  const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < count) {
    float c, s;
    bm_turn(start + j, c, s);
    co[j] = c;
    si[j] = s;
  }
}

// The objective of Sec. III-B for packed decisions, one wavefront per frame,
// in the fixed point of ngdbf_objective (exact, order-free int64 sums).
__global__ void objective_kernel(const uint16_t *t16, int off_rowptr, int dc, int n, int m,
                                 const void *y, int y_format, float ymax, const uint8_t *bits,
                                 int64_t n_frames, int64_t *out) {
  const int lane = threadIdx.x % kWave;
  const int64_t f = (int64_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
  if (f >= n_frames) return;  // the whole wavefront leaves together
  const int nbytes = (n + 7) >> 3;
  const uint8_t *b = bits + f * nbytes;
  int64_t part = 0;
  for (int k = lane; k < n; k += kWave) {
    const float v = saturate(y_format == NGDBF_Y_I8 ? load_sample<NGDBF_Y_I8>(y, f * n + k)
                                                    : load_sample<NGDBF_Y_F32>(y, f * n + k),
                             ymax);
    const int64_t yf = fixed_sample(v);
    part += ((b[k >> 3] >> (k & 7)) & 1u) ? -yf : yf;
  }
  const uint16_t *rp = t16 + off_rowptr;
  for (int i = lane; i < m; i += kWave) {
    const int e0 = dc ? i * dc : rp[i], e1 = dc ? e0 + dc : rp[i + 1];
    uint32_t par = 0;
    for (int e = e0; e < e1; ++e) {
      const int k = t16[e];
      par ^= (b[k >> 3] >> (k & 7)) & 1u;
    }
    part += par ? -((int64_t)1 << 20) : ((int64_t)1 << 20);
  }
  part = wave_sum_i64(part);
  if (lane == 0) out[f] = part;
}

__global__ void probe_quad_kernel(uint32_t start, uint32_t count, uint64_t frame, uint32_t iter,
                                  uint32_t k0, uint32_t k1, float *out) {
  const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < count) {
    const Draw4 d = draw_quad(start + j, iter, frame, k0, k1);
    for (int b = 0; b < 4; ++b) out[4 * (size_t)j + b] = d.z[b];
  }
}

}  // namespace ngdbf

// ==================================================================== host

struct ngdbf_code {
  int32_t n, m, nnz;
  int device;
  uint32_t *d_tables;  // uint16 col_idx | row_idx [| row_ptr | col_ptr], dword padded
  int32_t table_words;
  int32_t off_row, off_rowptr, off_colptr;
  int32_t dv, dc;      // uniform degrees (0 if irregular)
  int32_t max_col_deg, max_row_deg;
  int32_t shape[3];    // fixed launch shape (waves/frame, quads/lane, frames/block), 0 = default
  uint64_t *stats;     // device counters of the settle test, or NULL
};

namespace {

thread_local char g_err[512] = "";

ngdbf_status fail(int code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
ngdbf_status fail(int code, const char *fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof g_err, fmt, ap);
  va_end(ap);
  return (ngdbf_status)code;
}

ngdbf_status ok() {
  g_err[0] = '\0';
  return NGDBF_OK;
}

// an internal status as the ABI's type
ngdbf_status st(int rc) { return (ngdbf_status)rc; }

}  // namespace

namespace ngdbf_host {
// message of a failed call of another translation unit (the server runtime)
int set_error(int code, const char *msg) {
  snprintf(g_err, sizeof g_err, "%s", msg);
  return code;
}

int fail(int code, const char *fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof g_err, fmt, ap);
  va_end(ap);
  return code;
}
}  // namespace ngdbf_host

namespace {

using ngdbf_host::Shape;

// ---------------------------------------------------------------- devices

// Frame queues: every launch takes one queue (ngdbf::kQueueWords counters:
// the runs handed out per queue lane, the takers that have finished); its
// last taker sets them back to zero, so a launch finds its queue zero whether
// it runs directly or replayed from a captured graph.  Direct launches take
// queues from a ring of kQueueSlots, launches recorded into a graph from a
// ring of kCapturedSlots of their own, so that a graph's queues are never
// those of direct launches running beside its replays.  Launches in flight
// together take different queues: an event recorded after each direct launch
// marks its queue free again, a launch passes over ring slots that are still
// held, and one that finds all of them held fails with NGDBF_EBUSY instead of
// sharing one.  A graph must not be replayed on two streams at the same time.
constexpr int kQueueSlots = 1024;
constexpr int kCapturedSlots = 1024;

struct DeviceState {
  int cus = 0;
  // kQueueSlots + kCapturedSlots queues, allocated with the first code
  unsigned long long *queues = nullptr;
  // one event per direct-ring queue, recorded on the launch's stream after it
  std::vector<hipEvent_t> queue_done;
  std::atomic<uint32_t> next_queue{0};     // direct launches
  std::atomic<uint32_t> next_captured{0};  // launches recorded under stream capture
  std::mutex mu;                      // guards the fork/join pool below
  std::vector<hipStream_t> streams;   // library streams for batched jobs
  std::vector<hipEvent_t> events;     // one per stream, plus the fork event
  hipEvent_t fork = nullptr;
};

DeviceState &device_state(int dev) {
  static std::mutex mu;
  static std::vector<DeviceState *> all;
  std::lock_guard<std::mutex> g(mu);
  if ((int)all.size() <= dev) all.resize(dev + 1, nullptr);
  if (!all[dev]) {
    all[dev] = new DeviceState();  // lives until the process ends
    hipDeviceProp_t p;
    if (hipGetDeviceProperties(&p, dev) == hipSuccess) all[dev]->cus = p.multiProcessorCount;
  }
  return *all[dev];
}

}  // namespace

int ngdbf_host::device_cus(int dev) { return device_state(dev).cus; }

// ------------------------------------------------- allocation-free decode

namespace ngdbf {
// Device scratch of ngdbf_decode_noalloc: one frame queue (kQueueWords
// counters, 1152 bytes) in a static array, which every device that loads the
// library holds until the process ends.  Every call on a device shares it.
constexpr size_t kScratchWords = (size_t)kQueueWords;
static __device__ __align__(256) unsigned long long scratch[kScratchWords];
}  // namespace ngdbf

namespace {

// The device address of `scratch` on device dev (the device current), looked
// up once per device.  In host code the array's name is only a stand-in for
// the symbol, never a device address: kernels and fills get this pointer.
int scratch_address(int dev, unsigned long long **out) {
  static std::mutex mu;
  static std::vector<unsigned long long *> addr;
  std::lock_guard<std::mutex> g(mu);
  if ((int)addr.size() <= dev) addr.resize((size_t)dev + 1, nullptr);
  if (!addr[(size_t)dev]) {
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(ngdbf::scratch));
    if (e != hipSuccess || !ptr)
      return fail(NGDBF_EDEVICE, "scratch symbol address on device %d: %s", dev, hipGetErrorString(e));
    addr[(size_t)dev] = (unsigned long long *)ptr;
  }
  *out = addr[(size_t)dev];
  return NGDBF_OK;
}

}  // namespace

namespace {

// allocate (and zero) the device's frame queues once; not inside a capture
int ensure_queues(int dev) {
  static std::mutex mu;
  std::lock_guard<std::mutex> g(mu);
  DeviceState &st = device_state(dev);
  if (st.queues) return NGDBF_OK;
  const size_t bytes =
      (size_t)(kQueueSlots + kCapturedSlots) * ngdbf::kQueueWords * sizeof(unsigned long long);
  unsigned long long *q = nullptr;
  if (hipMalloc((void **)&q, bytes) != hipSuccess)
    return fail(NGDBF_ENOMEM, "device allocation of the frame queues failed");
  if (hipMemset(q, 0, bytes) != hipSuccess || hipDeviceSynchronize() != hipSuccess) {
    (void)hipFree(q);
    return fail(NGDBF_EDEVICE, "clearing the frame queues failed");
  }
  std::vector<hipEvent_t> evs((size_t)kQueueSlots, nullptr);
  for (auto &e : evs) {
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
      for (auto &e2 : evs)
        if (e2) (void)hipEventDestroy(e2);
      (void)hipFree(q);
      return fail(NGDBF_EDEVICE, "cannot create the frame queue events");
    }
  }
  st.queue_done = std::move(evs);
  st.queues = q;  // kept until the process ends
  return NGDBF_OK;
}

// The queue of the next launch: ring slot *slot (-1 for a captured launch,
// whose graph replays the device cannot see from here).  A direct-ring slot
// whose previous launch has not finished is refused (NGDBF_EBUSY).
int take_queue(int dev, bool captured, unsigned long long **queue, int *slot) {
  DeviceState &st = device_state(dev);
  if (!st.queues) return fail(NGDBF_EDEVICE, "no frame queues on device %d", dev);
  if (captured) {
    const uint32_t i = (uint32_t)kQueueSlots + st.next_captured.fetch_add(1u) % (uint32_t)kCapturedSlots;
    *queue = st.queues + (size_t)ngdbf::kQueueWords * i;
    *slot = -1;
    return NGDBF_OK;
  }
  // An earlier error is left for the caller to report (the slot is then taken
  // unchecked).  A slot whose launch is still running is passed over: one long
  // launch may hold its queue while a thousand short ones on other streams
  // come and go.  Every probe draws a fresh ring index, so a slot goes to two
  // takers only if a full turn of the ring passes between them.
  const bool check = hipPeekAtLastError() == hipSuccess;
  for (int probe = 0; probe < kQueueSlots; ++probe) {
    const uint32_t i = st.next_queue.fetch_add(1u) % (uint32_t)kQueueSlots;
    if (check) {
      const hipError_t q = hipEventQuery(st.queue_done[i]);
      if (q == hipErrorNotReady) {
        (void)hipGetLastError();  // "not ready" is not an error
        continue;
      }
      if (q != hipSuccess) return fail(NGDBF_EDEVICE, "frame queue event: %s", hipGetErrorString(q));
    }
    *queue = st.queues + (size_t)ngdbf::kQueueWords * i;
    *slot = (int)i;
    return NGDBF_OK;
  }
  return fail(NGDBF_EBUSY, "all %d frame queues of device %d are held by launches in flight",
              kQueueSlots, dev);
}

// mark a direct launch's queue as held until the work queued on s so far ends
int hold_queue(int dev, int slot, hipStream_t s) {
  if (slot < 0) return NGDBF_OK;
  if (hipEventRecord(device_state(dev).queue_done[(size_t)slot], s) != hipSuccess)
    return fail(NGDBF_EDEVICE, "frame queue event record failed");
  return NGDBF_OK;
}

// Whether work queued on `s` now is recorded into a graph.  With an earlier
// error pending nothing is asked (the caller reports that error next); an
// error of the query itself (the legacy stream during a global capture)
// counts as "not capturing" and is cleared.
bool stream_capturing(hipStream_t s) {
  if (hipPeekAtLastError() != hipSuccess) return false;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &cs) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return cs == hipStreamCaptureStatusActive;
}

}  // namespace

namespace {

// ---------------------------------------------------------------- shapes

// (waves per frame, quads per lane) pairs with built kernels
#define NGDBF_PAIR(W_, Q_) {W_, Q_},
constexpr int kShapes[][2] = {NGDBF_SHAPES(NGDBF_PAIR)};
#undef NGDBF_PAIR

bool shape_built(int wpf, int qpl) {
  for (const auto &sh : kShapes)
    if (sh[0] == wpf && sh[1] == qpl) return true;
  return false;
}

// What a launch keeps in LDS besides the code tables.
struct Layout {
  bool trace = false;   // flip-mask row per frame
  bool ext = false;     // extended decoder: two 64-bit reduction words
  int stream_len = 0;   // noise-reuse samples per frame
  bool lists = true;    // per-wave Box-Muller lists (the settle-test path)
  bool packed = false;  // quantized multi-bit decoder with noise reuse in 16-bit lanes
  bool lazy = true;     // the base decoder: thresholds from a table and flip counts
  bool bounded = false; // single-bit flips with per-bit draws (argmin by bounds)
  bool one_flip = false; // single-bit rule: one flip, at most a column degree of toggles, per round
  int thr_words = 0;    // the base decoder's table theta lambda^u, u = 0..T (float)
  int t_max = 0;
};

// int16 samples in the packed decoder's reversed stream: L, then zeros up to a
// multiple of four covering the last quad's two 8-byte words (L + 7)
int packed_stream_lr(const Layout &L) { return L.stream_len > 0 ? (L.stream_len + 8 + 3) & ~3 : 0; }
// words of the packed decoder's threshold table theta~(u), u = 0..T (int16)
int packed_table_words(const Layout &L) { return L.packed ? ((L.t_max + 2) / 2 + 1) & ~1 : 0; }

int list_words(const Layout &L) {
  if (!L.lists) return 0;
  return L.lazy ? ngdbf::kEntryWordsLazy * ngdbf::kListCapLazy + ngdbf::kDecisionWords
                : ngdbf::kEntryWords * ngdbf::kListCap;
}

// Word offsets within one frame slot: s | u | x | flips | count | 2 event
// counters | 2 count changes | toggles | events [| flip counts] [| reductions
// | stream]; even,
// so that 64-bit LDS atomics are aligned.
struct SlotPlan {
  int red_off = 0, stream_off = 0, clear_words = 0, slot_words = 0, fc_off = 0;
};

// Check-toggle events a frame lists per round for the parallel u update: up
// to one per check (a round toggles each check at most once), 256 per frame
// (events past the cap are applied by their owners, slower but alike; busy
// rounds list nothing where the owners apply their events themselves, and a
// small list leaves C4000's frames the LDS for five frames per CU), within
// the exact range of the kernel's division by d_c; irregular codes apply
// their toggles directly and list none.
int event_cap(const ngdbf_code *c, int wpf, bool one_flip) {
  (void)wpf;
  if (!c->dc) return 0;
  const int cap = std::min(std::min(c->m, 256), std::min(4095, ((1 << 20) - 1) / (c->dc * c->dc)));
  return one_flip ? std::min(cap, 16) : cap;  // one flip toggles at most d_v <= 15 checks
}

// Rounds that start with more unsatisfied checks than this list no events:
// the owner of each byte of s applies its toggled checks' d_c updates of u
// itself.  That pays where the checks give every other lane of the frame a
// byte to own and rows are light (d_c <= 8) and the round is busy; light
// rounds and heavy rows list their events and spread the updates over all
// lanes.
constexpr uint32_t kListUnsatMax = 64;
uint32_t list_unsat_max(const ngdbf_code *c, int wpf) {
  if (c->dc && c->dc <= 8 && (c->m + 7) / 8 >= 32 * wpf) return kListUnsatMax;
  return 0xFFFFFFFFu;
}

SlotPlan slot_plan(const ngdbf_code *c, const Layout &L, int wpf) {
  int w = (c->m + 31) / 32 + (c->n + 3) / 4 + ((c->n + 31) / 32) * (L.trace ? 2 : 1) + 5 +
          (c->m + 31) / 32 + event_cap(c, wpf, L.one_flip);
  SlotPlan p;
  if (L.ext) {
    w = (w + 1) & ~1;
    p.red_off = w;
    w += 4;
    p.stream_off = w;
    p.clear_words = w;
    if (L.packed)
      w += packed_stream_lr(L) / 2;       // one int16 row
    else
      w += 4 * ((L.stream_len + 3) / 4);  // four interleaved rows
  } else {
    if (L.lazy) {
      // flip counts of every bit of every quad: 8-bit if T <= 255, else 16-bit
      p.fc_off = w;
      w += (L.t_max <= 255 ? 1 : 2) * ((c->n + 3) / 4);
    }
    p.clear_words = w;
  }
  p.slot_words = (w + 1) & ~1;
  return p;
}

// The base kernel with two or more waves per frame reads the code tables
// from global memory (the kernel's TG); every other instance stages them.
bool tables_in_lds(const Layout &L, const Shape &sh) { return !(L.lazy && sh.wpf >= 2); }

// LDS words: [code tables] | [threshold table] | frame slots | wave lists
int qtab_offset(const ngdbf_code *c, const Layout &L, const Shape &sh) {
  return tables_in_lds(L, sh) ? (c->table_words + 1) & ~1 : 0;
}
int slots_offset(const ngdbf_code *c, const Layout &L, const Shape &sh) {
  return qtab_offset(c, L, sh) + ((packed_table_words(L) + L.thr_words + 1) & ~1);
}

size_t lds_bytes(const ngdbf_code *c, const Shape &sh, const Layout &L) {
  return ((size_t)slots_offset(c, L, sh) + (size_t)sh.fpb * slot_plan(c, L, sh.wpf).slot_words +
          (size_t)(sh.block() / 64) * list_words(L)) * 4;
}

// The base decoder keeps its threshold table theta lambda^u (u = 0..T) in
// LDS; a longer adaptive schedule runs in the extended multi-bit kernel,
// which keeps one threshold per bit in registers.
constexpr int kLazyMaxT = 8191;

bool extended(const ngdbf_params *p) {
  return p->variant != NGDBF_MULTI || p->quant_bits != 0 || p->noise_reuse != 0 ||
         (p->lambda != 1.0f && p->t_max > kLazyMaxT);
}

// The quantized multi-bit decoder with noise reuse runs in packed 16-bit lanes
// (its threshold table of T + 1 entries lives in LDS, so T is bounded).
constexpr int kPackedMaxT = 4095;
bool packed_decoder(const ngdbf_params *p) {
  return p->variant == NGDBF_MULTI && p->quant_bits != 0 && p->noise_reuse != 0 &&
         p->t_max <= kPackedMaxT;
}

Layout layout_of(const ngdbf_code *c, const ngdbf_params *p, bool trace) {
  Layout L;
  L.trace = trace;
  L.ext = extended(p);
  L.stream_len = (p->noise_reuse && p->t_max > 0) ? c->n + p->t_max - 1 : 0;
  // the lists serve rounds with per-bit draws (the multi-bit settle test, the
  // single-bit candidates)
  L.lists = !p->noise_reuse;
  L.packed = packed_decoder(p);
  L.lazy = !L.ext;
  L.bounded = p->variant == NGDBF_SINGLE && !p->noise_reuse;
  L.one_flip = p->variant == NGDBF_SINGLE;
  L.thr_words = (L.lazy && p->lambda != 1.0f) ? p->t_max + 1 : 0;
  L.t_max = p->t_max;
  return L;
}

// NGDBF_OK if the shape can decode the code, else an error with a message
int check_shape(const ngdbf_code *c, const Shape &sh, const Layout &L) {
  const int nq = (c->n + 3) / 4;
  if (!shape_built(sh.wpf, sh.qpl))
    return fail(NGDBF_EUNSUPPORTED, "no kernel for %d waves x %d quads", sh.wpf, sh.qpl);
  if (nq > 64 * sh.wpf * sh.qpl)
    return fail(NGDBF_EINVAL, "%d waves x %d quads hold %d quads, the code has %d", sh.wpf,
                sh.qpl, 64 * sh.wpf * sh.qpl, nq);
  if (sh.wpf > 1 && sh.fpb != 1)
    return fail(NGDBF_EINVAL, "a frame of several waves is a workgroup of its own");
  if (sh.fpb < 1 || sh.block() > 1024)
    return fail(NGDBF_EINVAL, "workgroup of %d threads", sh.block());
  // (the kernel adds a few bytes of static LDS: the workgroup's frame index)
  if (lds_bytes(c, sh, L) > 160 * 1024 - 256)
    return fail(NGDBF_EUNSUPPORTED, "shape needs %zu B of LDS", lds_bytes(c, sh, L));
  return NGDBF_OK;
}

// The code's fixed shape, or the default: the fewest waves per frame, then
// the fewest quads per lane that hold the code (at most two quads per lane
// for the extended decoders); sixteen single-wave frames per workgroup (or
// as many as the LDS holds), which then share one copy of the code tables.
int pick_shape(const ngdbf_code *c, const Layout &L, Shape *out) {
  if (c->shape[0]) {
    *out = Shape{c->shape[0], c->shape[1], c->shape[2]};
    return check_shape(c, *out, L);
  }
  const int nq = (c->n + 3) / 4;
  // the extended decoders keep more per-bit state: at most two quads per
  // lane (more waves per frame) keeps them out of register spills (the packed
  // quantized decoder holds two bits per register and needs no such limit;
  // the single-bit decoder by bounds runs faster with one wave per frame,
  // which saves its frame-wide reductions their barriers)
  const bool few_quads = L.ext && !L.packed && !L.bounded;
  // the base kernel's frames of more than one wave read the code tables from
  // global memory (more workgroups per CU); for codes above 1024 bits the
  // fewest waves that hold the code win (C2048 at (2, 4) in 199 ms against
  // 216 at (4, 2) on a mixed-SNR batch)
  for (const auto &sh : kShapes) {
    if (few_quads && sh[1] > 2 && nq <= 64 * 16) continue;
    if (nq <= 64 * sh[0] * sh[1]) {
      // frames per workgroup: 16, 12, 8, 4, 2, 1 (one if a frame takes several waves)
      Shape cand{sh[0], sh[1], sh[0] == 1 ? 16 : 1};
      while (check_shape(c, cand, L) != NGDBF_OK && cand.fpb > 1)
        cand.fpb = cand.fpb == 16 ? 12 : (cand.fpb == 12 ? 8 : cand.fpb / 2);
      if (check_shape(c, cand, L) == NGDBF_OK) {
        *out = cand;
        return ok();
      }
    }
  }
  return fail(NGDBF_EUNSUPPORTED, "no launch shape fits n = %d", c->n);
}

int check_params(const ngdbf_params *p) {
  if (!p) return fail(NGDBF_EINVAL, "params is NULL");
  if (!(p->w > 0.0f) || !std::isfinite(p->w)) return fail(NGDBF_EINVAL, "w must be finite and > 0");
  if (!std::isfinite(p->theta)) return fail(NGDBF_EINVAL, "theta must be finite");
  if (!(p->lambda > 0.0f && p->lambda <= 1.0f))
    return fail(NGDBF_EINVAL, "lambda must be in (0, 1]");
  if (!(p->eta >= 0.0f) || !std::isfinite(p->eta)) return fail(NGDBF_EINVAL, "eta must be finite and >= 0");
  if (std::isnan(p->ymax)) return fail(NGDBF_EINVAL, "ymax is NaN");
  if (p->t_max < 0 || p->t_max > 65535) return fail(NGDBF_EINVAL, "t_max must be in [0, 65535]");
  if (p->smooth_window < 0) return fail(NGDBF_EINVAL, "smooth_window must be >= 0");
  if (p->smooth_window > 0 && std::min(p->smooth_window, p->t_max) >= 32767)
    return fail(NGDBF_EUNSUPPORTED, "smoothing over more than 32767 rounds");
  if (p->y_format != NGDBF_Y_F32 && p->y_format != NGDBF_Y_I8)
    return fail(NGDBF_EINVAL, "unknown y_format %d", p->y_format);
  if (p->variant < NGDBF_MULTI || p->variant > NGDBF_MODE_SWITCH)
    return fail(NGDBF_EINVAL, "unknown variant %d", p->variant);
  if (p->quant_bits < 0 || p->quant_bits > 8)
    return fail(NGDBF_EINVAL, "quant_bits must be in [0, 8]");
  if (p->quant_bits && !(p->ymax > 0.0f && std::isfinite(p->ymax)))
    return fail(NGDBF_EINVAL, "the quantizer needs a finite ymax > 0");
  if (p->quant_bits && p->variant == NGDBF_MODE_SWITCH)
    return fail(NGDBF_EINVAL, "mode switching is defined for the binary32 decoder only");
  if (p->noise_reuse != 0 && p->noise_reuse != 1)
    return fail(NGDBF_EINVAL, "noise_reuse must be 0 or 1");
  return NGDBF_OK;
}

// g(v) of Sec. IV-E in half-step units (the device's quant_half, for the
// weight, which is quantized once per launch)
float quant_half_host(float v, float c, float top) {
  if (v == 0.0f) return 0.0f;
  float L = std::floor(std::fabs(v) * c);
  L = (L > top) ? top : L;
  const float mag = 2.0f * L + 1.0f;
  return v < 0.0f ? -mag : mag;
}

// Everything a launch needs, validated on the host before any device work.
struct Prepared {
  ngdbf::DecodeArgs a;
  Shape sh;
  size_t lds;
  int dev;
  int queue_slot;  // direct-ring slot of the launch's queue, -1 if captured
  int y_format;
  bool ext;
  bool packed;
};

int prepare(const ngdbf_code *code, const void *y, int64_t n_frames, const float *sigma,
            float sigma_scalar, const ngdbf_params *p, uint64_t seed, uint64_t frame_base,
            uint8_t *out_bits, int32_t *out_iters, uint8_t *out_conv, uint8_t *trace,
            const Shape *force, Prepared *out, bool captured, const ngdbf_segment *segments = nullptr,
            int32_t n_segments = 0, int64_t pool_frames = -1,
            unsigned long long *fixed_queue = nullptr) {
  // host-side validation, parameters first (no device state is touched)
  int rc = check_params(p);
  if (rc) return rc;
  if (n_frames < 0) return fail(NGDBF_EINVAL, "n_frames < 0");
  if (!sigma && (!(sigma_scalar >= 0.0f) || !std::isfinite(sigma_scalar)))
    return fail(NGDBF_EINVAL, "sigma_scalar must be finite and >= 0");
  if (!code) return fail(NGDBF_EINVAL, "code is NULL");
  if (n_frames > 0 && (!y || !out_bits || !out_iters))
    return fail(NGDBF_EINVAL, "y, out_bits and out_iters are required");
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return fail(NGDBF_EDEVICE, "no HIP device");
  if (dev != code->device)
    return fail(NGDBF_EINVAL, "code lives on device %d, current device is %d", code->device, dev);
  const Layout L = layout_of(code, p, trace != nullptr);
  Shape sh;
  if (force) {
    sh = *force;
    rc = check_shape(code, sh, L);
  } else {
    rc = pick_shape(code, L, &sh);
  }
  if (rc) return rc;
  const int n = code->n, m = code->m;
  ngdbf::DecodeArgs &a = out->a;
  a.tables = code->d_tables;
  a.table_words = code->table_words;
  a.off_row = code->off_row;
  a.off_rowptr = code->off_rowptr;
  a.off_colptr = code->off_colptr;
  a.dv = code->dv;
  a.dc = code->dc;
  a.n = n;
  a.m = m;
  a.y = y;
  a.n_frames = n_frames;
  a.sigma = sigma;
  a.sigma_scalar = sigma_scalar;
  a.w = p->w;
  a.theta = p->theta;
  a.lambda = p->lambda;
  a.eta = p->eta;
  a.ymax = p->ymax;
  a.t_max = p->t_max;
  a.smooth_window = p->smooth_window;
  a.key0 = (uint32_t)seed;
  a.key1 = (uint32_t)(seed >> 32);
  a.frame_base = frame_base;
  a.out_bits = out_bits;
  a.out_iters = out_iters;
  a.out_conv = out_conv;
  a.trace = trace;
  a.segments = segments;
  a.n_segments = n_segments;
  a.pool_frames = pool_frames >= 0 ? pool_frames : n_frames;
  a.frames_per_block = sh.fpb;
  a.sw_words = (m + 31) / 32;
  a.uw_words = (n + 3) / 4;
  a.xw_words = (n + 31) / 32;
  const SlotPlan plan = slot_plan(code, L, sh.wpf);
  a.dc_recip = code->dc ? (uint32_t)(((1u << 20) + code->dc - 1) / code->dc) : 0u;
  a.event_cap = event_cap(code, sh.wpf, L.one_flip);
  a.list_unsat_max = list_unsat_max(code, sh.wpf);
  a.slot_words = plan.slot_words;
  a.slots_off = slots_offset(code, L, sh);
  a.qtab_off = qtab_offset(code, L, sh);
  a.thr_off = qtab_offset(code, L, sh);
  a.fc_off = plan.fc_off;
  a.fc_bytes = p->t_max <= 255 ? 1 : 0;
  a.stats = code->stats;
  if (fixed_queue) {
    a.queue = fixed_queue;
    out->queue_slot = -1;
  } else {
    rc = take_queue(dev, captured, &a.queue, &out->queue_slot);
    if (rc) return rc;
  }
  a.stream_lr = packed_stream_lr(L);
  a.red_off = plan.red_off;
  a.stream_off = plan.stream_off;
  a.clear_words = plan.clear_words;
  a.stream_len = L.stream_len;
  a.stream_q = (L.stream_len + 3) / 4;
  a.list_words = list_words(L);
  a.variant = p->variant;
  a.quant_bits = p->quant_bits;
  a.noise_reuse = p->noise_reuse;
  if (p->quant_bits) {
    const int nq_levels = 1 << p->quant_bits;
    a.qc = (float)nq_levels / (2.0f * p->ymax);   // fl32(N_Q / 2 Y_max)
    a.qtop = (float)(nq_levels / 2 - 1);
    a.wq = quant_half_host(p->w, a.qc, a.qtop);
    a.qbound = (float)(nq_levels - 1);
  } else {
    a.qc = a.qtop = a.wq = a.qbound = 0.0f;
  }
  out->sh = sh;
  out->lds = lds_bytes(code, sh, L);
  out->dev = dev;
  out->y_format = p->y_format;
  out->ext = L.ext;
  out->packed = L.packed;
  return ok();
}

int launch_prepared(const Prepared &pr, hipStream_t s) {
  const bool trace = pr.a.trace != nullptr;
  using ngdbf_host::dispatch;
  if (pr.ext) {
    if (pr.a.variant == NGDBF_SINGLE)
      return ngdbf_host::dispatch_ext_single(pr.sh, pr.a, pr.lds, pr.dev, s, pr.y_format, trace);
    if (pr.a.variant == NGDBF_MODE_SWITCH)
      return ngdbf_host::dispatch_ext_switch(pr.sh, pr.a, pr.lds, pr.dev, s, pr.y_format, trace);
    if (pr.packed)
      return ngdbf_host::dispatch_ext_packed(pr.sh, pr.a, pr.lds, pr.dev, s, pr.y_format, trace);
    return ngdbf_host::dispatch_ext_multi(pr.sh, pr.a, pr.lds, pr.dev, s, pr.y_format, trace);
  }
  constexpr int kBase = ngdbf::kExtNone;
  if (pr.y_format == NGDBF_Y_I8) {
    return trace ? dispatch<NGDBF_Y_I8, true, kBase>(pr.sh, pr.a, pr.lds, pr.dev, s)
                 : dispatch<NGDBF_Y_I8, false, kBase>(pr.sh, pr.a, pr.lds, pr.dev, s);
  }
  return trace ? dispatch<NGDBF_Y_F32, true, kBase>(pr.sh, pr.a, pr.lds, pr.dev, s)
               : dispatch<NGDBF_Y_F32, false, kBase>(pr.sh, pr.a, pr.lds, pr.dev, s);
}

// launch, then hold the launch's queue until it has run
int enqueue(const Prepared &pr, hipStream_t s) {
  if (pr.a.n_frames == 0) return ok();
  const int rc = launch_prepared(pr, s);
  if (rc) return rc;
  return hold_queue(pr.dev, pr.queue_slot, s);
}

int pending_error() {
  // report an earlier asynchronous fault before queueing more work
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(NGDBF_EDEVICE, "earlier HIP error: %s", hipGetErrorString(e));
  return NGDBF_OK;
}

int decode_common(const ngdbf_code *code, const void *y, int64_t n_frames, const float *sigma,
                  float sigma_scalar, const ngdbf_params *p, uint64_t seed, uint64_t frame_base,
                  uint8_t *out_bits, int32_t *out_iters, uint8_t *out_conv, uint8_t *trace,
                  void *stream) {
  hipStream_t s = (hipStream_t)stream;
  Prepared pr;
  int rc = prepare(code, y, n_frames, sigma, sigma_scalar, p, seed, frame_base, out_bits,
                   out_iters, out_conv, trace, nullptr, &pr, stream_capturing(s));
  if (rc) return rc;
  rc = pending_error();
  if (rc) return rc;
  if (trace && n_frames > 0 && p->t_max > 0) {
    const size_t tb = (size_t)n_frames * (size_t)p->t_max * (size_t)((code->n + 7) / 8);
    const size_t blocks = std::min<size_t>((tb + 255) / 256, 4096);
    hipLaunchKernelGGL(ngdbf::clear_bytes_kernel, dim3((unsigned)blocks), dim3(256), 0, s, trace, tb);
    if (hipGetLastError() != hipSuccess) return fail(NGDBF_EDEVICE, "trace clear failed");
  }
  return enqueue(pr, s);
}

}  // namespace

extern "C" {

const char *ngdbf_last_error(void) { return g_err; }

ngdbf_status ngdbf_create_code(int32_t n, int32_t m, int64_t nnz, const int32_t *row_ptr,
                               const int32_t *col_idx, ngdbf_code **out) {
  if (!out) return fail(NGDBF_EINVAL, "out is NULL");
  *out = nullptr;
  if (!row_ptr || !col_idx) return fail(NGDBF_EINVAL, "row_ptr and col_idx are required");
  if (m < 1 || n <= m || n > 65535) return fail(NGDBF_EINVAL, "need 1 <= m < n <= 65535");
  if (nnz < m) return fail(NGDBF_EINVAL, "nnz = %lld: every one of the %d rows needs an edge", (long long)nnz, m);
  if (nnz > (1 << 24)) return fail(NGDBF_EUNSUPPORTED, "nnz %lld exceeds 2^24", (long long)nnz);
  if (row_ptr[0] != 0) return fail(NGDBF_EINVAL, "row_ptr[0] must be 0");
  for (int i = 0; i < m; ++i) {
    if (row_ptr[i + 1] <= row_ptr[i]) return fail(NGDBF_EINVAL, "row %d is empty or row_ptr decreases", i);
    if (row_ptr[i + 1] > nnz) return fail(NGDBF_EINVAL, "row_ptr[%d] = %d exceeds nnz = %lld", i + 1, row_ptr[i + 1], (long long)nnz);
  }
  if (row_ptr[m] != nnz)
    return fail(NGDBF_EINVAL, "row_ptr[m] = %d differs from nnz = %lld", row_ptr[m], (long long)nnz);
  std::vector<int32_t> colcnt(n + 1, 0);
  for (int i = 0; i < m; ++i) {
    for (int e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
      const int c = col_idx[e];
      if (c < 0 || c >= n) return fail(NGDBF_EINVAL, "col_idx[%d] = %d out of range", e, c);
      for (int e2 = row_ptr[i]; e2 < e; ++e2)
        if (col_idx[e2] == c) return fail(NGDBF_EINVAL, "row %d repeats column %d", i, c);
      colcnt[c + 1]++;
    }
  }
  for (int k = 0; k < n; ++k)
    if (colcnt[k + 1] == 0) return fail(NGDBF_EINVAL, "column %d is empty", k);
  std::vector<int32_t> colptr(n + 1, 0);
  for (int k = 0; k < n; ++k) colptr[k + 1] = colptr[k] + colcnt[k + 1];
  std::vector<int32_t> rowidx(nnz), fill(colptr.begin(), colptr.end() - 1);
  for (int i = 0; i < m; ++i)
    for (int e = row_ptr[i]; e < row_ptr[i + 1]; ++e) rowidx[fill[col_idx[e]]++] = i;

  int maxr = 0, maxc = 0, minr = 1 << 30, minc = 1 << 30;
  for (int i = 0; i < m; ++i) {
    maxr = std::max(maxr, row_ptr[i + 1] - row_ptr[i]);
    minr = std::min(minr, row_ptr[i + 1] - row_ptr[i]);
  }
  for (int k = 0; k < n; ++k) {
    maxc = std::max(maxc, colptr[k + 1] - colptr[k]);
    minc = std::min(minc, colptr[k + 1] - colptr[k]);
  }
  if (maxc > 15) return fail(NGDBF_EUNSUPPORTED, "column degree %d exceeds 15", maxc);
  const bool regular = (maxr == minr) && (maxc == minc);
  if (nnz > 65535 && !regular)
    return fail(NGDBF_EUNSUPPORTED, "an irregular code needs nnz <= 65535 (16-bit pointers)");
  // uint16 tables: col_idx | row_idx [| row_ptr | col_ptr]
  std::vector<uint16_t> t16;
  t16.reserve((size_t)(2 * nnz + m + n + 4));
  for (int64_t e = 0; e < nnz; ++e) t16.push_back((uint16_t)col_idx[e]);
  const int off_row = (int)t16.size();
  for (int64_t e = 0; e < nnz; ++e) t16.push_back((uint16_t)rowidx[e]);
  int off_rowptr = 0, off_colptr = 0;
  if (!regular) {
    off_rowptr = (int)t16.size();
    for (int i = 0; i <= m; ++i) t16.push_back((uint16_t)row_ptr[i]);
    off_colptr = (int)t16.size();
    for (int k = 0; k <= n; ++k) t16.push_back((uint16_t)colptr[k]);
  }
  if (t16.size() & 1) t16.push_back(0);
  const int words = (int)(t16.size() / 2);

  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return fail(NGDBF_EDEVICE, "no HIP device");
  ngdbf_code *c = (ngdbf_code *)calloc(1, sizeof(ngdbf_code));
  if (!c) return fail(NGDBF_ENOMEM, "host allocation failed");
  c->n = n;
  c->m = m;
  c->nnz = (int32_t)nnz;
  c->device = dev;
  c->table_words = words;
  c->off_row = off_row;
  c->off_rowptr = off_rowptr;
  c->off_colptr = off_colptr;
  c->dv = regular ? maxc : 0;
  c->dc = regular ? maxr : 0;
  c->max_row_deg = maxr;
  c->max_col_deg = maxc;
  c->shape[0] = c->shape[1] = c->shape[2] = 0;
  const size_t bytes = (size_t)words * 4;
  if (int qrc = ensure_queues(dev)) {
    free(c);
    return st(qrc);
  }
  if (hipMalloc((void **)&c->d_tables, bytes) != hipSuccess) {
    free(c);
    return fail(NGDBF_ENOMEM, "device allocation of %zu bytes failed", bytes);
  }
  if (hipMemcpy(c->d_tables, t16.data(), bytes, hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipFree(c->d_tables);
    free(c);
    return fail(NGDBF_EDEVICE, "upload of the code tables failed");
  }
  *out = c;
  return ok();
}

ngdbf_status ngdbf_destroy_code(ngdbf_code *code) {
  if (!code) return ok();
  const hipError_t e = hipFree(code->d_tables);
  free(code);
  if (e != hipSuccess) return fail(NGDBF_EDEVICE, "hipFree failed: %s", hipGetErrorString(e));
  return ok();
}

ngdbf_status ngdbf_code_info(const ngdbf_code *code, int32_t *n, int32_t *m, int32_t *nnz) {
  if (!code) return fail(NGDBF_EINVAL, "code is NULL");
  if (n) *n = code->n;
  if (m) *m = code->m;
  if (nnz) *nnz = code->nnz;
  return ok();
}

ngdbf_status ngdbf_decode(const ngdbf_code *code, const void *y, int64_t n_frames, const float *sigma,
                 float sigma_scalar, const ngdbf_params *params, uint64_t seed,
                 uint64_t frame_base, uint8_t *out_bits, int32_t *out_iters,
                 uint8_t *out_converged, void *stream) {
  return st(decode_common(code, y, n_frames, sigma, sigma_scalar, params, seed, frame_base, out_bits,
                          out_iters, out_converged, nullptr, stream));
}

ngdbf_status ngdbf_decode_trace(const ngdbf_code *code, const void *y, int64_t n_frames, const float *sigma,
                       float sigma_scalar, const ngdbf_params *params, uint64_t seed,
                       uint64_t frame_base, uint8_t *out_bits, int32_t *out_iters,
                       uint8_t *out_converged, uint8_t *flip_masks, void *stream) {
  if (n_frames > 0 && params && params->t_max > 0 && !flip_masks)
    return fail(NGDBF_EINVAL, "flip_masks is required");
  return st(decode_common(code, y, n_frames, sigma, sigma_scalar, params, seed, frame_base, out_bits,
                          out_iters, out_converged, flip_masks ? flip_masks : nullptr, stream));
}

ngdbf_status ngdbf_decode_noalloc(const ngdbf_code *code, const void *y, int64_t n_frames,
                                  const float *sigma, float sigma_scalar,
                                  const ngdbf_params *params, uint64_t seed, uint64_t frame_base,
                                  uint8_t *out_bits, int32_t *out_iters, uint8_t *out_converged,
                                  void *stream) {
  hipStream_t s = (hipStream_t)stream;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return fail(NGDBF_EDEVICE, "no HIP device");
  unsigned long long *q = nullptr;
  int rc = scratch_address(dev, &q);
  if (rc) return st(rc);
  // the launch needs one queue; nothing else of it depends on the batch size
  static_assert(ngdbf::kScratchWords >= (size_t)ngdbf::kQueueWords, "scratch holds one queue");
  const size_t need = (size_t)ngdbf::kQueueWords * sizeof(unsigned long long);
  if (need > sizeof(ngdbf::scratch))
    return fail(NGDBF_EUNSUPPORTED, "the launch needs %zu bytes of scratch, the library holds %zu",
                need, sizeof(ngdbf::scratch));
  Prepared pr;
  rc = prepare(code, y, n_frames, sigma, sigma_scalar, params, seed, frame_base, out_bits, out_iters,
               out_converged, nullptr, nullptr, &pr, false, nullptr, 0, -1, q);
  if (rc) return st(rc);
  rc = pending_error();
  if (rc) return st(rc);
  if (n_frames == 0) return ok();
  // the queue's counters start at zero (the last launch's final taker also
  // clears them, but a launch that never ran to its end would not have)
  hipLaunchKernelGGL(ngdbf::clear_bytes_kernel, dim3(1), dim3(256), 0, s, (uint8_t *)q, need);
  if (hipGetLastError() != hipSuccess) return fail(NGDBF_EDEVICE, "scratch clear failed");
  return st(launch_prepared(pr, s));
}

ngdbf_status ngdbf_noise_probe(int32_t kind, uint32_t start, uint32_t count, uint64_t seed, uint64_t frame,
                      uint32_t iter, float *out0, float *out1, void *stream) {
  if (count == 0) return ok();
  if (!out0) return fail(NGDBF_EINVAL, "out0 is NULL");
  hipStream_t s = (hipStream_t)stream;
  const unsigned blocks = (count + 255) / 256;
  if (kind == 0) {
    if (start < 1 || (uint64_t)start + count - 1 > (1ull << 24))
      return fail(NGDBF_EINVAL, "radius probe range must lie in [1, 2^24]");
    hipLaunchKernelGGL(ngdbf::probe_radius_kernel, dim3(blocks), dim3(256), 0, s, start, count, out0);
  } else if (kind == 1) {
    if (!out1) return fail(NGDBF_EINVAL, "out1 is NULL");
    if ((uint64_t)start + count > (1ull << 24))
      return fail(NGDBF_EINVAL, "angle probe range must lie in [0, 2^24)");
    hipLaunchKernelGGL(ngdbf::probe_turn_kernel, dim3(blocks), dim3(256), 0, s, start, count, out0,
                       out1);
  } else if (kind == 2) {
    hipLaunchKernelGGL(ngdbf::probe_quad_kernel, dim3(blocks), dim3(256), 0, s, start, count, frame,
                       iter, (uint32_t)seed, (uint32_t)(seed >> 32), out0);
  } else {
    return fail(NGDBF_EINVAL, "unknown probe kind %d", kind);
  }
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(NGDBF_EDEVICE, "probe launch failed: %s", hipGetErrorString(e));
  return ok();
}

ngdbf_status ngdbf_objective(const ngdbf_code *code, const void *y, int32_t y_format, int64_t n_frames,
                    float ymax, const uint8_t *bits, int64_t *out, void *stream) {
  if (!code) return fail(NGDBF_EINVAL, "code is NULL");
  if (n_frames < 0) return fail(NGDBF_EINVAL, "n_frames < 0");
  if (y_format != NGDBF_Y_F32 && y_format != NGDBF_Y_I8)
    return fail(NGDBF_EINVAL, "unknown y_format %d", y_format);
  if (n_frames == 0) return ok();
  if (!y || !bits || !out) return fail(NGDBF_EINVAL, "y, bits and out are required");
  int rc = pending_error();
  if (rc) return st(rc);
  const int per_block = 4;  // frames (wavefronts) per workgroup
  const int64_t blocks = (n_frames + per_block - 1) / per_block;
  if (blocks > 0x7FFFFFFF) return fail(NGDBF_EINVAL, "too many frames for one launch");
  hipLaunchKernelGGL(ngdbf::objective_kernel, dim3((unsigned)blocks), dim3(64 * per_block), 0,
                     (hipStream_t)stream, (const uint16_t *)code->d_tables, code->off_rowptr,
                     code->dc, code->n, code->m, y, y_format, ymax, bits, n_frames, out);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(NGDBF_EDEVICE, "launch failed: %s", hipGetErrorString(e));
  return ok();
}

ngdbf_status ngdbf_decode_segments(const ngdbf_code *code, const void *y_pool, const float *sigma_pool,
                          float sigma_scalar, int64_t pool_frames, const ngdbf_params *params,
                          const ngdbf_segment *segments, int32_t n_segments, int64_t n_frames,
                          uint8_t *bits_pool, int32_t *iters_pool, uint8_t *conv_pool,
                          void *stream) {
  if (n_frames > 0 && (n_segments < 1 || !segments))
    return fail(NGDBF_EINVAL, "segments are required");
  if (pool_frames < 0) return fail(NGDBF_EINVAL, "pool_frames < 0");
  Prepared pr;
  int rc = prepare(code, y_pool, n_frames, sigma_pool, sigma_scalar, params, 0, 0, bits_pool,
                   iters_pool, conv_pool, nullptr, nullptr, &pr, stream_capturing((hipStream_t)stream),
                   segments, n_segments, pool_frames);
  if (rc) return st(rc);
  rc = pending_error();
  if (rc) return st(rc);
  return st(enqueue(pr, (hipStream_t)stream));
}

ngdbf_status ngdbf_code_set_shape(ngdbf_code *code, int32_t waves_per_frame, int32_t quads_per_lane,
                         int32_t frames_per_block) {
  if (!code) return fail(NGDBF_EINVAL, "code is NULL");
  if (!waves_per_frame && !quads_per_lane && !frames_per_block) {
    code->shape[0] = code->shape[1] = code->shape[2] = 0;
    return ok();
  }
  const Shape sh{waves_per_frame, quads_per_lane, frames_per_block};
  int rc = check_shape(code, sh, Layout{});
  if (rc) return st(rc);
  code->shape[0] = sh.wpf;
  code->shape[1] = sh.qpl;
  code->shape[2] = sh.fpb;
  return ok();
}

ngdbf_status ngdbf_code_set_stats(ngdbf_code *code, uint64_t *counters) {
  if (!code) return fail(NGDBF_EINVAL, "code is NULL");
  code->stats = counters;
  return ok();
}

ngdbf_status ngdbf_code_get_shape(const ngdbf_code *code, const ngdbf_params *params, int32_t shape[3]) {
  if (!code || !shape) return fail(NGDBF_EINVAL, "code and shape are required");
  if (params) {
    if (int rc = check_params(params)) return st(rc);
  }
  Shape sh;
  int rc = pick_shape(code, params ? layout_of(code, params, false) : Layout{}, &sh);
  if (rc) return st(rc);
  shape[0] = sh.wpf;
  shape[1] = sh.qpl;
  shape[2] = sh.fpb;
  return ok();
}

ngdbf_status ngdbf_autotune(ngdbf_code *code, const void *y, int64_t n_frames, const float *sigma,
                   float sigma_scalar, const ngdbf_params *params, uint64_t seed, int32_t best[3],
                   float *elapsed_ms, void *stream) {
  if (!code) return fail(NGDBF_EINVAL, "code is NULL");
  if (n_frames <= 0) return fail(NGDBF_EINVAL, "autotuning needs a sample of frames");
  if (int prc = check_params(params)) return st(prc);
  int rc = pending_error();
  if (rc) return st(rc);
  hipStream_t s = (hipStream_t)stream;
  const size_t nb = (size_t)(code->n + 7) / 8;
  uint8_t *bits = nullptr;
  int32_t *iters = nullptr;
  if (hipMalloc((void **)&bits, (size_t)n_frames * nb) != hipSuccess ||
      hipMalloc((void **)&iters, (size_t)n_frames * 4) != hipSuccess) {
    (void)hipFree(bits);
    return fail(NGDBF_ENOMEM, "autotune scratch of %lld frames", (long long)n_frames);
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  (void)hipEventCreate(&e0);
  (void)hipEventCreate(&e1);
  Shape best_sh{0, 0, 0};
  float best_ms = 0.0f;
  const int nq = (code->n + 3) / 4;
  for (const auto &ks : kShapes) {
    if (nq > 64 * ks[0] * ks[1]) continue;
    // more quads per lane or waves per frame than the code needs only idle lanes
    if (ks[1] > 1 && nq <= 64 * ks[0] * (ks[1] / 2)) continue;
    if (ks[0] > 1 && nq <= 64 * (ks[0] / 2) * ks[1]) continue;
    for (int fpb : {1, 2, 4, 8, 12, 16}) {
      const Shape cand{ks[0], ks[1], fpb};
      if (check_shape(code, cand, layout_of(code, params, false)) != NGDBF_OK) continue;
      Prepared pr;
      rc = prepare(code, y, n_frames, sigma, sigma_scalar, params, seed, 0, bits, iters, nullptr,
                   nullptr, &cand, &pr, false);
      if (rc) break;
      rc = enqueue(pr, s);  // warm-up
      if (rc == NGDBF_EUNSUPPORTED) {  // rejected before launch (occupancy, LDS)
        rc = NGDBF_OK;
        continue;
      }
      if (rc) break;
      (void)hipEventRecord(e0, s);
      for (int rep = 0; rep < 2 && !rc; ++rep) rc = enqueue(pr, s);
      (void)hipEventRecord(e1, s);
      if (rc) break;
      if (hipEventSynchronize(e1) != hipSuccess) {
        rc = fail(NGDBF_EDEVICE, "autotune run failed");
        break;
      }
      float ms = 0.0f;
      (void)hipEventElapsedTime(&ms, e0, e1);
      ms *= 0.5f;
      if (!best_sh.wpf || ms < best_ms) {
        best_sh = cand;
        best_ms = ms;
      }
    }
    if (rc) break;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipFree(bits);
  (void)hipFree(iters);
  if (rc) return st(rc);
  if (!best_sh.wpf) return fail(NGDBF_EUNSUPPORTED, "no launch shape fits this code");
  code->shape[0] = best_sh.wpf;
  code->shape[1] = best_sh.qpl;
  code->shape[2] = best_sh.fpb;
  if (best) {
    best[0] = best_sh.wpf;
    best[1] = best_sh.qpl;
    best[2] = best_sh.fpb;
  }
  if (elapsed_ms) *elapsed_ms = best_ms;
  return ok();
}

ngdbf_status ngdbf_decode_batch(const ngdbf_job *jobs, int32_t n_jobs, void *stream) {
  if (n_jobs < 0 || (n_jobs > 0 && !jobs)) return fail(NGDBF_EINVAL, "bad job array");
  // the library streams join a capture of `stream` through the fork event
  const bool captured = n_jobs > 0 && stream_capturing((hipStream_t)stream);
  // every job takes its own frame queue before any is launched: a batch may
  // not wrap its ring
  if (n_jobs > (captured ? kCapturedSlots : kQueueSlots))
    return fail(NGDBF_EINVAL, "%d jobs exceed the %d frame queues of one batch", n_jobs,
                captured ? kCapturedSlots : kQueueSlots);
  std::vector<Prepared> prs((size_t)n_jobs);
  for (int i = 0; i < n_jobs; ++i) {
    const ngdbf_job &j = jobs[i];
    const int rc = prepare(j.code, j.y, j.n_frames, j.sigma, j.sigma_scalar, &j.params, j.seed,
                           j.frame_base, j.out_bits, j.out_iters, j.out_converged, nullptr,
                           nullptr, &prs[i], captured);
    if (rc) {
      char msg[512];
      snprintf(msg, sizeof msg, "%s", g_err);
      return fail(rc, "job %d: %s", i, msg);
    }
    if (i && prs[i].dev != prs[0].dev) return fail(NGDBF_EINVAL, "jobs span several devices");
  }
  int rc = pending_error();
  if (rc) return st(rc);
  hipStream_t s = (hipStream_t)stream;
  if (n_jobs == 0) return ok();
  if (n_jobs == 1) return st(enqueue(prs[0], s));
  // A job of kFullJob frames or more fills the device by itself (its
  // persistent grid is the resident capacity): such jobs run one after another
  // on `stream`; the smaller ones run concurrently beside them on library
  // streams, forked from and joined back to `stream`.
  constexpr int64_t kFullJob = 65536;
  std::vector<int> small, large;
  for (int i = 0; i < n_jobs; ++i) (prs[i].a.n_frames >= kFullJob ? large : small).push_back(i);
  if (small.empty()) {
    for (int i : large) {
      rc = enqueue(prs[i], s);
      if (rc) return st(rc);
    }
    return ok();
  }
  DeviceState &ds = device_state(prs[0].dev);
  std::lock_guard<std::mutex> g(ds.mu);
  const size_t lanes = std::min(small.size(), (size_t)8);
  while (ds.streams.size() < lanes) {
    hipStream_t ns = nullptr;
    hipEvent_t ne = nullptr;
    // default priority: library streams never outrank the caller's work
    if (hipStreamCreateWithFlags(&ns, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&ne, hipEventDisableTiming) != hipSuccess)
      return fail(NGDBF_EDEVICE, "cannot create the batch streams");
    ds.streams.push_back(ns);
    ds.events.push_back(ne);
  }
  if (!ds.fork && hipEventCreateWithFlags(&ds.fork, hipEventDisableTiming) != hipSuccess)
    return fail(NGDBF_EDEVICE, "cannot create the fork event");
  // fork: every library stream waits for the work already queued on `stream`
  if (hipEventRecord(ds.fork, s) != hipSuccess) return fail(NGDBF_EDEVICE, "fork record failed");
  for (size_t l = 0; l < lanes; ++l)
    if (hipStreamWaitEvent(ds.streams[l], ds.fork, 0) != hipSuccess)
      return fail(NGDBF_EDEVICE, "fork wait failed");
  for (size_t q = 0; q < small.size() && !rc; ++q)
    rc = enqueue(prs[(size_t)small[q]], ds.streams[q % lanes]);
  for (size_t q = 0; q < large.size() && !rc; ++q) rc = enqueue(prs[(size_t)large[q]], s);
  // join: `stream` waits for every library stream (also after a failure, so
  // that the fork/join structure stays balanced under graph capture)
  for (size_t l = 0; l < lanes; ++l) {
    if (hipEventRecord(ds.events[l], ds.streams[l]) != hipSuccess ||
        hipStreamWaitEvent(s, ds.events[l], 0) != hipSuccess)
      return fail(NGDBF_EDEVICE, "join failed");
  }
  return st(rc);
}

}  // extern "C"
