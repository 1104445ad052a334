// The checking stand-in for the HIP runtime declared in fakehip/hip/hip_runtime.h.
// One device (0).  Device memory is host memory, registered per allocation;
// every copy and every simulated kernel checks its ranges against the live
// allocations.  Work queued on a stream runs later, in stream order: when the
// host synchronises the stream or an event recorded on it, when it frees
// memory (hipFree waits for the device), or, for an event query, sometimes.
// Streams are drained in a random interleaving.  Calls that a stream capture
// forbids (synchronous copies, waits, allocation) end the run when a capture
// is open in the calling thread.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <random>
#include <string>
#include <vector>

struct FakeOp {
  std::string what;
  std::function<void()> fn;
};

struct FakeGraph {
  bool live = true;
  std::vector<FakeOp> ops;
};

struct FakeGraphExec {
  bool live = true;
  std::vector<FakeOp> ops;
};

struct FakeStream {
  bool live = true;
  bool capturing = false;
  bool thread_local_capture = false;
  FakeGraph* cap = nullptr;
  std::deque<FakeOp> q;
  uint64_t enq = 0, done = 0;  // operations queued and run so far
};

struct FakeEvent {
  bool live = true;
  bool timing = true;
  bool recorded = false;
  FakeStream* s = nullptr;
  uint64_t seq = 0;  // complete once s->done >= seq
};

namespace {

enum Kind { kDevice, kPinned, kSymbol };
struct Alloc {
  size_t bytes;
  Kind kind;
};

std::recursive_mutex g_mu;
std::map<uintptr_t, Alloc> g_allocs;  // live allocations by base address
std::vector<std::unique_ptr<FakeStream>> g_streams;
std::vector<std::unique_ptr<FakeEvent>> g_events;
std::vector<std::unique_ptr<FakeGraph>> g_graphs;
std::vector<std::unique_ptr<FakeGraphExec>> g_execs;
FakeStream g_null;
std::mt19937_64 g_rng(12345);
thread_local int t_device = 0;
thread_local int t_captures = 0;  // thread-local-mode captures open in this thread

[[noreturn]] void fail(const char* fmt, const char* a, const void* p = nullptr, size_t n = 0) {
  std::fprintf(stdout, "fakehip violation: ");
  std::fprintf(stdout, fmt, a, p, n);
  std::fprintf(stdout, "\n");
  std::fflush(stdout);
  std::_Exit(3);
}

FakeStream* S(hipStream_t s) { return s ? s : &g_null; }

const Alloc* find(const void* p, size_t bytes, uintptr_t* base_out = nullptr) {
  const uintptr_t x = (uintptr_t)p;
  auto it = g_allocs.upper_bound(x);
  if (it == g_allocs.begin()) return nullptr;
  --it;
  if (x < it->first || x + bytes > it->first + it->second.bytes || x + bytes < x) return nullptr;
  if (base_out) *base_out = it->first;
  return &it->second;
}

void no_capture(const char* what) {
  if (t_captures) fail("%s called while a stream capture is open in this thread", what);
}

void run_one(FakeStream* s) {
  FakeOp op = std::move(s->q.front());
  s->q.pop_front();
  op.fn();
  ++s->done;
}

void run_until(FakeStream* s, uint64_t seq) {
  while (s->done < seq) {
    if (s->q.empty()) fail("%s: stream has fewer operations than an event expects", "run_until");
    run_one(s);
  }
}

void drain_all() {
  for (;;) {
    std::vector<FakeStream*> busy;
    if (!g_null.q.empty()) busy.push_back(&g_null);
    for (auto& s : g_streams)
      if (!s->q.empty()) busy.push_back(s.get());
    if (busy.empty()) return;
    run_one(busy[g_rng() % busy.size()]);
  }
}

bool is_dev_kind(const Alloc* a) { return a && a->kind != kPinned; }

}  // namespace

namespace fakehip {

void enqueue(hipStream_t s, const char* what, std::function<void()> op) {
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  FakeStream* st = S(s);
  if (!st->live) fail("%s: queued on a destroyed stream", what);
  if (st->capturing) {
    st->cap->ops.push_back(FakeOp{what, std::move(op)});
    return;
  }
  st->q.push_back(FakeOp{what, std::move(op)});
  ++st->enq;
}

bool is_device(const void* p, size_t bytes) {
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  return is_dev_kind(find(p, bytes ? bytes : 1));
}

void need_device(const void* p, size_t bytes, const char* what) {
  if (bytes == 0) return;
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  if (!is_dev_kind(find(p, bytes)))
    fail("%s: [%p, +%zu) is not inside a live device allocation", what, p, bytes);
}

void drain() {
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  drain_all();
}

size_t live_device_allocations() {
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  size_t n = 0;
  for (auto& kv : g_allocs) n += kv.second.kind != kSymbol;
  return n;
}

size_t live_streams() {
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  size_t n = 0;
  for (auto& s : g_streams) n += s->live;
  return n;
}

size_t live_events() {
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  size_t n = 0;
  for (auto& e : g_events) n += e->live;
  return n;
}

}  // namespace fakehip

hipError_t hipGetDevice(int* dev) {
  *dev = t_device;
  return hipSuccess;
}

hipError_t hipSetDevice(int dev) {
  if (dev != 0) return hipErrorInvalidValue;
  t_device = dev;
  return hipSuccess;
}

hipError_t hipGetDeviceProperties(hipDeviceProp_t* prop, int dev) {
  if (dev != 0) return hipErrorInvalidValue;
  std::memset(prop, 0, sizeof(*prop));
  std::strcpy(prop->name, "fake MI355X");
  std::strcpy(prop->gcnArchName, "gfx950:sramecc+:xnack-");
  prop->multiProcessorCount = 256;
  return hipSuccess;
}

hipError_t hipMalloc(void** p, size_t bytes) {
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  no_capture("hipMalloc");
  if (!p) return hipErrorInvalidValue;
  void* m = std::malloc(bytes ? bytes : 1);
  if (!m) return hipErrorOutOfMemory;
  std::memset(m, 0xCD, bytes);  // device memory starts with no defined contents
  g_allocs[(uintptr_t)m] = Alloc{bytes ? bytes : 1, kDevice};
  *p = m;
  return hipSuccess;
}

hipError_t hipFree(void* p) {
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  no_capture("hipFree");
  if (!p) return hipSuccess;
  drain_all();  // hipFree waits for the device
  auto it = g_allocs.find((uintptr_t)p);
  if (it == g_allocs.end() || it->second.kind != kDevice)
    fail("%s: %p is not the base of a live device allocation", "hipFree", p);
  g_allocs.erase(it);
  std::free(p);
  return hipSuccess;
}

hipError_t hipHostMalloc(void** p, size_t bytes, unsigned) {
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  no_capture("hipHostMalloc");
  void* m = std::malloc(bytes ? bytes : 1);
  if (!m) return hipErrorOutOfMemory;
  g_allocs[(uintptr_t)m] = Alloc{bytes ? bytes : 1, kPinned};
  *p = m;
  return hipSuccess;
}

hipError_t hipHostFree(void* p) {
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  no_capture("hipHostFree");
  if (!p) return hipSuccess;
  drain_all();
  auto it = g_allocs.find((uintptr_t)p);
  if (it == g_allocs.end() || it->second.kind != kPinned)
    fail("%s: %p is not the base of a live pinned allocation", "hipHostFree", p);
  g_allocs.erase(it);
  std::free(p);
  return hipSuccess;
}

static void check_copy(void* dst, const void* src, size_t bytes, hipMemcpyKind kind,
                       const char* what) {
  if (bytes == 0) return;
  const Alloc* ad = find(dst, bytes);
  const Alloc* as = find(src, bytes);
  const bool dd = is_dev_kind(ad), sd = is_dev_kind(as);
  switch (kind) {
    case hipMemcpyHostToDevice:
      if (!dd) fail("%s: destination [%p, +%zu) is not device memory", what, dst, bytes);
      if (sd) fail("%s: source [%p, +%zu) is device memory", what, src, bytes);
      break;
    case hipMemcpyDeviceToHost:
      if (!sd) fail("%s: source [%p, +%zu) is not device memory", what, src, bytes);
      if (dd) fail("%s: destination [%p, +%zu) is device memory", what, dst, bytes);
      break;
    case hipMemcpyDeviceToDevice:
      if (!dd || !sd) fail("%s: [%p, +%zu) device-to-device outside device memory", what, dst, bytes);
      break;
    case hipMemcpyDefault: {
      // a device-looking pointer must be a whole live range
      uintptr_t b;
      for (const void* p : {(const void*)dst, src})
        if (find(p, 1, &b) && !find(p, bytes))
          fail("%s: [%p, +%zu) runs past its allocation", what, p, bytes);
      break;
    }
    default: fail("%s: bad copy kind", what);
  }
}

hipError_t hipMemcpy(void* dst, const void* src, size_t bytes, hipMemcpyKind kind) {
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  no_capture("hipMemcpy");
  // a blocking copy on the null stream: earlier null-stream work first
  run_until(&g_null, g_null.enq);
  check_copy(dst, src, bytes, kind, "hipMemcpy");
  if (bytes) std::memmove(dst, src, bytes);
  return hipSuccess;
}

hipError_t hipMemcpyAsync(void* dst, const void* src, size_t bytes, hipMemcpyKind kind,
                          hipStream_t s) {
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  check_copy(dst, src, bytes, kind, "hipMemcpyAsync (at enqueue)");
  fakehip::enqueue(s, "hipMemcpyAsync", [=] {
    check_copy(dst, src, bytes, kind, "hipMemcpyAsync (when it runs)");
    if (bytes) std::memmove(dst, src, bytes);
  });
  return hipSuccess;
}

hipError_t hipMemset(void* p, int v, size_t bytes) {
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  no_capture("hipMemset");
  run_until(&g_null, g_null.enq);
  fakehip::need_device(p, bytes, "hipMemset");
  std::memset(p, v, bytes);
  return hipSuccess;
}

hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned) {
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  g_streams.emplace_back(new FakeStream);
  *s = g_streams.back().get();
  return hipSuccess;
}

hipError_t hipStreamDestroy(hipStream_t s) {
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  if (!s || !s->live) fail("%s: destroying a stream that is not live", "hipStreamDestroy");
  if (s->capturing) fail("%s: destroying a capturing stream", "hipStreamDestroy");
  while (!s->q.empty()) run_one(s);  // queued work still completes
  s->live = false;
  return hipSuccess;
}

hipError_t hipStreamSynchronize(hipStream_t s) {
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  no_capture("hipStreamSynchronize");
  FakeStream* st = S(s);
  if (!st->live) fail("%s: stream is not live", "hipStreamSynchronize");
  while (!st->q.empty()) run_one(st);
  return hipSuccess;
}

hipError_t hipDeviceSynchronize(void) {
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  no_capture("hipDeviceSynchronize");
  drain_all();
  return hipSuccess;
}

hipError_t hipStreamBeginCapture(hipStream_t s, hipStreamCaptureMode mode) {
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  if (!s || !s->live || s->capturing) return hipErrorInvalidValue;
  s->capturing = true;
  s->thread_local_capture = mode != hipStreamCaptureModeRelaxed;
  if (s->thread_local_capture) ++t_captures;
  g_graphs.emplace_back(new FakeGraph);
  s->cap = g_graphs.back().get();
  return hipSuccess;
}

hipError_t hipStreamEndCapture(hipStream_t s, hipGraph_t* g) {
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  if (!s || !s->capturing) return hipErrorInvalidValue;
  s->capturing = false;
  if (s->thread_local_capture) --t_captures;
  *g = s->cap;
  s->cap = nullptr;
  return hipSuccess;
}

hipError_t hipGraphInstantiate(hipGraphExec_t* e, hipGraph_t g, hipGraphNode_t*, char*, size_t) {
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  if (!g || !g->live) return hipErrorInvalidValue;
  g_execs.emplace_back(new FakeGraphExec);
  g_execs.back()->ops = g->ops;
  *e = g_execs.back().get();
  return hipSuccess;
}

hipError_t hipGraphLaunch(hipGraphExec_t e, hipStream_t s) {
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  if (!e || !e->live) fail("%s: graph exec is not live", "hipGraphLaunch");
  for (const FakeOp& op : e->ops) fakehip::enqueue(s, op.what.c_str(), op.fn);
  return hipSuccess;
}

hipError_t hipGraphExecDestroy(hipGraphExec_t e) {
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  if (!e || !e->live) fail("%s: graph exec is not live", "hipGraphExecDestroy");
  e->live = false;
  e->ops.clear();
  return hipSuccess;
}

hipError_t hipGraphDestroy(hipGraph_t g) {
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  if (!g || !g->live) fail("%s: graph is not live", "hipGraphDestroy");
  g->live = false;
  g->ops.clear();
  return hipSuccess;
}

hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned flags) {
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  g_events.emplace_back(new FakeEvent);
  g_events.back()->timing = !(flags & hipEventDisableTiming);
  *e = g_events.back().get();
  return hipSuccess;
}

hipError_t hipEventCreate(hipEvent_t* e) { return hipEventCreateWithFlags(e, 0); }

hipError_t hipEventDestroy(hipEvent_t e) {
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  if (!e || !e->live) fail("%s: event is not live", "hipEventDestroy");
  e->live = false;
  return hipSuccess;
}

hipError_t hipEventRecord(hipEvent_t e, hipStream_t s) {
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  if (!e || !e->live) fail("%s: event is not live", "hipEventRecord");
  FakeStream* st = S(s);
  if (!st->live) fail("%s: stream is not live", "hipEventRecord");
  if (st->capturing) fail("%s: recorded into a capturing stream", "hipEventRecord");
  e->recorded = true;
  e->s = st;
  e->seq = st->enq;
  return hipSuccess;
}

hipError_t hipEventSynchronize(hipEvent_t e) {
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  no_capture("hipEventSynchronize");
  if (!e || !e->live) fail("%s: event is not live", "hipEventSynchronize");
  if (e->recorded) run_until(e->s, e->seq);
  return hipSuccess;
}

hipError_t hipEventQuery(hipEvent_t e) {
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  no_capture("hipEventQuery");
  if (!e || !e->live) fail("%s: event is not live", "hipEventQuery");
  if (!e->recorded || e->s->done >= e->seq) return hipSuccess;
  if (g_rng() & 1) run_one(e->s);  // the device makes progress now and then
  return e->s->done >= e->seq ? hipSuccess : hipErrorNotReady;
}

hipError_t hipEventElapsedTime(float* ms, hipEvent_t a, hipEvent_t b) {
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  if (!ms || !a || !b || !a->live || !b->live) return hipErrorInvalidHandle;
  if (!a->timing || !b->timing || !a->recorded || !b->recorded) return hipErrorInvalidHandle;
  if (a->s->done < a->seq || b->s->done < b->seq) return hipErrorNotReady;
  *ms = 0.001f * (float)(b->seq >= a->seq ? b->seq - a->seq + 1 : 1);
  return hipSuccess;
}

hipError_t hipGetSymbolAddress(void** p, FakeSymbol sym) {
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  if (!p || !sym.addr) return hipErrorInvalidValue;
  if (!find(sym.addr, sym.bytes)) g_allocs[(uintptr_t)sym.addr] = Alloc{sym.bytes, kSymbol};
  *p = sym.addr;
  return hipSuccess;
}
