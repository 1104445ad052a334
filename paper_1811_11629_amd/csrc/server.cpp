// Continuous-batching server over a device-resident pool of instances.
//
// A background thread runs the request loop: admit waiting requests while the
// output arena (device memory owned by the server) and the continuation slots
// have room, plan the next chunk of every admitted request (Scheduler), and
// enqueue the chunks as one batched launch on the server's stream.  A request
// whose chunk ends inside a 2^20 block resumes in a later iteration from the
// chain state its last tile left on the device (message and skip at the
// boundary), so no index is computed twice; requests arriving meanwhile join
// at the next iteration.  Up to two iterations are in flight; an event per
// iteration marks the requests whose last chunk it ran.
#include <hip/hip_runtime.h>

#include <atomic>
#include <chrono>
#include <condition_variable>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>

#include "host_internal.h"
#include "scheduler.h"

using namespace rsaprng;

namespace {

using Clock = std::chrono::steady_clock;

constexpr uint32_t kSlots = 1u << 16;
constexpr int kDepth = 2;

struct Inflight {
  hipEvent_t ev = nullptr;
  std::vector<SrvReq*> finishing;
};

// Restores the calling thread's current device.
struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    (void)hipSetDevice(dev);
  }
  ~DeviceGuard() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

}  // namespace

struct rsaprng_server_s {
  rsaprng_pool_t pool = nullptr;
  int device = 0;
  rsaprng_server_opts opts;
  rsaprng_config cfg;
  Device* dev = nullptr;
  Scratch sc;
  hipStream_t stream = nullptr;
  uint64_t* arena_c = nullptr;
  double* arena_r = nullptr;
  ChainState* states = nullptr;
  u64h arena_elems = 0;
  std::unique_ptr<Scheduler> sched;

  std::mutex mu;
  std::condition_variable cv;
  std::deque<rsaprng_completion> completions;
  std::unordered_map<uint64_t, std::unique_ptr<SrvReq>> by_tag;
  std::deque<Inflight> inflight;
  std::vector<PlanIn> plan;
  std::vector<SrvReq*> finishing;
  std::vector<Chain> chains;

  std::atomic<bool> stop{false};
  std::atomic<int> error{RSAPRNG_OK};
  std::thread th;
  Clock::time_point t0;
  uint64_t iterations = 0, outputs = 0;

  double now() const { return std::chrono::duration<double>(Clock::now() - t0).count(); }
  ~rsaprng_server_s();
  int init();
  void loop();
  int launch_next();  // with mu held
  void reap();        // with mu held
};

rsaprng_server_s::~rsaprng_server_s() {
  stop = true;
  cv.notify_all();
  if (th.joinable()) th.join();
  DeviceGuard g(device);
  if (stream) (void)hipStreamSynchronize(stream);
  for (auto& f : inflight)
    if (f.ev) (void)hipEventDestroy(f.ev);
  if (arena_c) (void)hipFree(arena_c);
  if (arena_r) (void)hipFree(arena_r);
  if (states) (void)hipFree(states);
  if (stream) (void)hipStreamDestroy(stream);
}

int rsaprng_server_s::init() {
  t0 = Clock::now();
  cfg = config_for_pool(pool, &opts.cfg, kModeGenerate);
  if (!opts.iter_outputs) opts.iter_outputs = 1ull << 26;
  if (!opts.chunk_outputs) opts.chunk_outputs = 1ull << 22;
  if (!opts.max_queue) opts.max_queue = 1u << 20;
  arena_elems = opts.arena_bytes / 16;
  if (arena_elems == 0) return RSAPRNG_E_ARG;
  if (opts.policy != kSrvRoundRobin && opts.policy != kSrvShortestFirst) return RSAPRNG_E_ARG;
  sched.reset(new Scheduler(arena_elems, kSlots, tile_size(cfg), opts.iter_outputs,
                            opts.chunk_outputs, opts.policy));
  device = pool_device(pool);
  DeviceGuard g(device);
  int rc = device_get(&dev);
  if (rc) return rc;
  if ((rc = sc.init())) return rc;
  if (hipStreamCreateWithFlags(&stream, hipStreamNonBlocking) != hipSuccess) return RSAPRNG_E_HIP;
  if (hipMalloc(&arena_c, arena_elems * 8) != hipSuccess) return RSAPRNG_E_OOM;
  if (hipMalloc(&arena_r, arena_elems * 8) != hipSuccess) return RSAPRNG_E_OOM;
  if (hipMalloc(&states, (size_t)kSlots * sizeof(ChainState)) != hipSuccess) return RSAPRNG_E_OOM;
  th = std::thread([this] { loop(); });
  return RSAPRNG_OK;
}

// Plans and enqueues one iteration: 1 if launched, 0 if nothing to run, or a status.
int rsaprng_server_s::launch_next() {
  u64h total = 0;
  if (!sched->plan(plan, finishing, &total)) return 0;
  u64h ntiles = 0;
  int rc = plan_chains(plan.data(), plan.size(), cfg, kModeGenerate, chains, &ntiles);
  LeadIn li;
  if (!rc) rc = split_leadin(chains, cfg, kModeGenerate, &li);
  if (!rc && !chains.empty()) group_by_exponent(chains, cfg, kModeGenerate, &pool_host(pool, 0), &li);
  void* dch = nullptr;
  int slot = 0;
  if (!rc) rc = sc.upload(chains.data(), chains.size() * sizeof(Chain), stream, &dch, &slot);
  if (!rc)
    rc = enqueue_launch(dev, &sc, cfg, kModeGenerate, pool_dev(pool), (const Chain*)dch,
                        (uint32_t)chains.size(), ntiles, arena_c, arena_r, nullptr, 0, states,
                        stream, nullptr, nullptr, 0, &li);
  if (!rc) rc = sc.mark(slot, stream);
  Inflight f;
  if (!rc && hipEventCreateWithFlags(&f.ev, hipEventDisableTiming) != hipSuccess)
    rc = RSAPRNG_E_HIP;
  if (!rc && hipEventRecord(f.ev, stream) != hipSuccess) rc = RSAPRNG_E_HIP;
  if (rc) {
    if (f.ev) (void)hipEventDestroy(f.ev);
    return rc;
  }
  f.finishing = finishing;
  inflight.push_back(std::move(f));
  ++iterations;
  outputs += total;
  return 1;
}

// Retires the iterations that have finished, oldest first.
void rsaprng_server_s::reap() {
  while (!inflight.empty()) {
    Inflight& f = inflight.front();
    const hipError_t q = hipEventQuery(f.ev);
    if (q == hipErrorNotReady) break;
    (void)hipEventDestroy(f.ev);
    if (q != hipSuccess) {
      error = RSAPRNG_E_HIP;
      inflight.pop_front();
      continue;
    }
    const double t = now();
    for (SrvReq* r : f.finishing) {
      sched->finish(r, t);
      rsaprng_completion c;
      c.tag = r->tag;
      c.c = arena_c + r->off;
      c.r = arena_r + r->off;
      c.count = r->count;
      c.t_submit = r->t_submit;
      c.t_admit = r->t_admit;
      c.t_done = r->t_done;
      completions.push_back(c);
    }
    inflight.pop_front();
  }
}

void rsaprng_server_s::loop() {
  (void)hipSetDevice(device);
  std::unique_lock<std::mutex> lk(mu);
  while (!stop) {
    sched->admit(now());
    int launched = 0;
    if ((int)inflight.size() < kDepth && error == RSAPRNG_OK) {
      launched = launch_next();
      if (launched < 0) {
        error = launched;
        launched = 0;
      }
    }
    reap();
    if (launched) continue;
    if (inflight.empty()) {
      // idle: wake on submit or release
      cv.wait_for(lk, std::chrono::milliseconds(1));
    } else {
      lk.unlock();
      std::this_thread::sleep_for(std::chrono::microseconds(10));
      lk.lock();
    }
  }
}

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

int rsaprng_server_create(rsaprng_pool_t pool, const rsaprng_server_opts* opts,
                          rsaprng_server_t* out) {
  if (!pool || !opts || !out) return RSAPRNG_E_NULL;
  auto s = std::make_unique<rsaprng_server_s>();
  s->pool = pool;
  s->opts = *opts;
  int rc = s->init();
  if (rc) return rc;
  *out = s.release();
  return RSAPRNG_OK;
}

int rsaprng_server_submit(rsaprng_server_t s, uint32_t inst, uint64_t k0, uint64_t count,
                          uint64_t tag) {
  if (!s) return RSAPRNG_E_NULL;
  if (inst >= rsaprng_pool_size(s->pool) || count == 0) return RSAPRNG_E_ARG;
  if (count - 1 > ~0ull - k0) return RSAPRNG_E_RANGE;
  if (count > s->arena_elems) return RSAPRNG_E_RANGE;
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->error != RSAPRNG_OK) return s->error;
  if (s->sched->waiting() >= s->opts.max_queue) return RSAPRNG_E_BUSY;
  if (s->by_tag.count(tag)) return RSAPRNG_E_ARG;
  auto r = std::make_unique<SrvReq>();
  r->tag = tag;
  r->inst = inst;
  r->e = pool_host(s->pool, inst).e;
  r->k0 = k0;
  r->count = count;
  r->pos = k0;
  r->t_submit = s->now();
  s->sched->enqueue(r.get());
  s->by_tag[tag] = std::move(r);
  s->cv.notify_one();
  return RSAPRNG_OK;
}

int rsaprng_server_poll(rsaprng_server_t s, rsaprng_completion* out, size_t max) {
  if (!s || (max && !out)) return RSAPRNG_E_NULL;
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->error != RSAPRNG_OK) return s->error;
  size_t n = 0;
  while (n < max && !s->completions.empty()) {
    out[n++] = s->completions.front();
    s->completions.pop_front();
  }
  return (int)n;
}

int rsaprng_server_read(rsaprng_server_t s, uint64_t tag, uint64_t offset, uint64_t count,
                        uint64_t* dst_u64, double* dst_f64, void* stream) {
  if (!s) return RSAPRNG_E_NULL;
  const uint64_t* c;
  const double* r;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->by_tag.find(tag);
    if (it == s->by_tag.end() || it->second->state != kSrvDone) return RSAPRNG_E_ARG;
    const SrvReq& q = *it->second;
    if (offset > q.count || count > q.count - offset) return RSAPRNG_E_RANGE;
    c = s->arena_c + q.off + offset;
    r = s->arena_r + q.off + offset;
  }
  if (count == 0) return RSAPRNG_OK;
  DeviceGuard g(s->device);
  hipStream_t st = (hipStream_t)stream;
  if (dst_u64 && hipMemcpyAsync(dst_u64, c, count * 8, hipMemcpyDefault, st) != hipSuccess)
    return RSAPRNG_E_HIP;
  if (dst_f64 && hipMemcpyAsync(dst_f64, r, count * 8, hipMemcpyDefault, st) != hipSuccess)
    return RSAPRNG_E_HIP;
  return hipStreamSynchronize(st) == hipSuccess ? RSAPRNG_OK : RSAPRNG_E_HIP;
}

int rsaprng_server_release(rsaprng_server_t s, uint64_t tag) {
  if (!s) return RSAPRNG_E_NULL;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->by_tag.find(tag);
  if (it == s->by_tag.end() || it->second->state != kSrvDone) return RSAPRNG_E_ARG;
  s->sched->release(it->second.get());
  s->by_tag.erase(it);
  s->cv.notify_one();
  return RSAPRNG_OK;
}

double rsaprng_server_now(rsaprng_server_t s) { return s ? s->now() : 0.0; }

int rsaprng_server_stats(rsaprng_server_t s, uint64_t* iterations, uint64_t* outputs,
                         uint64_t* waiting, uint64_t* active) {
  if (!s) return RSAPRNG_E_NULL;
  std::lock_guard<std::mutex> lk(s->mu);
  if (iterations) *iterations = s->iterations;
  if (outputs) *outputs = s->outputs;
  if (waiting) *waiting = s->sched->waiting();
  if (active) *active = s->sched->active();
  return RSAPRNG_OK;
}

int rsaprng_server_replay(rsaprng_server_t s, size_t n, const uint32_t* inst, const uint64_t* k0,
                          const uint64_t* count, const double* t_arrival, double* t_admit,
                          double* t_done) {
  if (!s || (n && (!inst || !k0 || !count || !t_arrival))) return RSAPRNG_E_NULL;
  for (size_t i = 1; i < n; ++i)
    if (t_arrival[i] < t_arrival[i - 1]) return RSAPRNG_E_ARG;
  const double base = s->now();
  const uint64_t tag0 = 1ull << 63;  // replay tags: tag0 + index
  size_t next = 0, done = 0;
  std::vector<rsaprng_completion> buf(4096);
  while (done < n) {
    const double t = s->now() - base;
    while (next < n && t_arrival[next] <= t) {
      const int rc = rsaprng_server_submit(s, inst[next], k0[next], count[next], tag0 + next);
      if (rc == RSAPRNG_E_BUSY) break;
      if (rc) return rc;
      ++next;
    }
    const int got = rsaprng_server_poll(s, buf.data(), buf.size());
    if (got < 0) return got;
    for (int i = 0; i < got; ++i) {
      const uint64_t tag = buf[i].tag;
      if (tag < tag0 || tag - tag0 >= n) continue;  // not one of ours
      const size_t k = (size_t)(tag - tag0);
      if (t_admit) t_admit[k] = buf[i].t_admit - base;
      if (t_done) t_done[k] = buf[i].t_done - base;
      const int rc = rsaprng_server_release(s, tag);
      if (rc) return rc;
      ++done;
    }
    if (got == 0) std::this_thread::sleep_for(std::chrono::microseconds(10));
  }
  return RSAPRNG_OK;
}

int64_t rsaprng_server_simulate(const rsaprng_config* cfg, uint64_t arena_elems,
                                uint64_t iter_outputs, uint64_t chunk_outputs, int policy,
                                size_t n,
                                const uint64_t* k0, const uint64_t* count,
                                const uint64_t* arrive_iter, uint64_t hold_iters, uint64_t* log,
                                size_t max_log) {
  if (n && (!k0 || !count || !arrive_iter)) return RSAPRNG_E_NULL;
  if (arena_elems == 0) return RSAPRNG_E_ARG;
  if (policy != kSrvRoundRobin && policy != kSrvShortestFirst) return RSAPRNG_E_ARG;
  for (size_t i = 0; i < n; ++i) {
    if (count[i] == 0 || count[i] > arena_elems) return RSAPRNG_E_RANGE;
    if (count[i] - 1 > ~0ull - k0[i]) return RSAPRNG_E_RANGE;
    if (i && arrive_iter[i] < arrive_iter[i - 1]) return RSAPRNG_E_ARG;
  }
  const rsaprng_config c = resolve_config(cfg);
  Scheduler sch(arena_elems, kSlots, tile_size(c), iter_outputs ? iter_outputs : 1ull << 26,
                chunk_outputs ? chunk_outputs : 1ull << 22, policy);
  std::vector<SrvReq> reqs(n);
  std::deque<std::pair<uint64_t, SrvReq*>> held;  // (release iteration, request)
  std::vector<PlanIn> plan;
  std::vector<SrvReq*> fin;
  size_t next = 0, done = 0, nlog = 0;
  uint64_t it = 0;
  while (done < n) {
    while (!held.empty() && held.front().first <= it) {
      sch.release(held.front().second);
      held.pop_front();
    }
    while (next < n && arrive_iter[next] <= it) {
      SrvReq& r = reqs[next];
      r.tag = next;
      r.inst = (uint32_t)next;  // the log reports the request index here
      r.k0 = r.pos = k0[next];
      r.count = count[next];
      sch.enqueue(&r);
      ++next;
    }
    sch.admit((double)it);
    u64h total = 0;
    if (sch.plan(plan, fin, &total)) {
      for (const PlanIn& p : plan) {
        if (log && nlog < max_log) {
          uint64_t* w = log + 7 * nlog;
          w[0] = p.inst;
          w[1] = it;
          w[2] = p.k0;
          w[3] = p.count;
          w[4] = p.out_off;
          w[5] = p.flags;
          w[6] = p.slot;
        }
        ++nlog;
      }
      for (SrvReq* r : fin) {
        sch.finish(r, (double)it);
        held.emplace_back(it + 1 + hold_iters, r);
        ++done;
      }
      ++it;
    } else if (!held.empty()) {
      it = std::max<uint64_t>(it + 1, held.front().first);
    } else if (next < n) {
      it = std::max<uint64_t>(it + 1, arrive_iter[next]);
    } else {
      return RSAPRNG_E_ARG;  // waiting requests that can never be admitted
    }
  }
  return (int64_t)nlog;
}

void rsaprng_server_destroy(rsaprng_server_t s) { delete s; }

}  // extern "C"
