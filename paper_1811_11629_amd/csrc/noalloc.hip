// rsaprng_pool_generate_noalloc: rsaprng_pool_generate without any allocation,
// for callers that cannot allocate device memory.  Every piece of launch
// scratch -- the uploaded chain table, the chain starts and the tile arrays of
// the two-pass prefix -- lives in `scratch`, one fixed array of device memory
// per GPU, which the library takes its address of once per device
// (hipGetSymbolAddress) and keeps until the process ends.  The chain table is
// planned into fixed host arrays of this file and copied from there, so the
// entry point calls no hipMalloc, hipHostMalloc or other allocating routine,
// and the host side allocates nothing either.
//
// Every call on a GPU shares that GPU's scratch: calls on one stream are
// ordered and safe; calls that overlap on one GPU (different streams, no
// ordering between them) race on it.
#include <hip/hip_runtime.h>

#include <mutex>

#include "host_internal.h"
#include "plan_core.h"

namespace rsaprng {
namespace {

constexpr size_t kScratchBytes = RSAPRNG_NOALLOC_SCRATCH_BYTES;
constexpr u64h kMaxChains = RSAPRNG_NOALLOC_MAX_CHAINS;
constexpr int kMaxDevices = 8;
constexpr int kSlots = 2;  // chain-table upload slots, used in turn

// Layout of scratch (byte offsets):
//   [0, 256)        control block (only the one-pass form, never used here, touches it)
//   kOffChains      the chain tables of the kSlots upload slots, kMaxChains each
//   kOffCstart      chain starts, one per chain
//   kOffTiles       tile arrays (tile -> chain, tile skip, chunk sums and prefixes)
constexpr size_t kOffChains = 256;
constexpr size_t kOffCstart = kOffChains + (size_t)kSlots * kMaxChains * sizeof(Chain);
constexpr size_t kOffTiles = kOffCstart + (size_t)kMaxChains * sizeof(ChainStart);
static_assert(kOffTiles % 256 == 0 && kOffTiles < kScratchBytes, "scratch layout");
constexpr size_t kTileBytes = kScratchBytes - kOffTiles;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

struct PerDevice {
  bool ready = false;
  unsigned char* ptr = nullptr;  // this device's copy of scratch
  hipEvent_t ev[kSlots] = {};    // the last launch that read each slot's chain table
  bool recorded[kSlots] = {};
  int next = 0;
};
PerDevice g_dev[kMaxDevices];
std::mutex g_mu[kMaxDevices];
// Host staging of the chain tables, one pair of slots per device.
alignas(64) Chain g_stage[kMaxDevices][kSlots][kMaxChains];

// Once per device, with that device current.
int setup(PerDevice& pd) {
  if (pd.ready) return RSAPRNG_OK;
  void* p = nullptr;
  if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return RSAPRNG_E_HIP;
  for (int i = 0; i < kSlots; ++i) {
    if (!pd.ev[i] && hipEventCreateWithFlags(&pd.ev[i], hipEventDisableTiming) != hipSuccess) {
      pd.ev[i] = nullptr;
      return RSAPRNG_E_HIP;
    }
  }
  pd.ptr = static_cast<unsigned char*>(p);
  pd.ready = true;
  return RSAPRNG_OK;
}

bool misaligned8(const void* p) { return p && ((uintptr_t)p & 7); }

}  // namespace
}  // namespace rsaprng

using namespace rsaprng;

extern "C" int rsaprng_pool_generate_noalloc(rsaprng_pool_t pool, const rsaprng_pool_req* reqs,
                                             size_t nreq, uint64_t* out_u64, double* out_f64,
                                             const rsaprng_config* cfg, void* stream) {
  if (!pool || (nreq && !reqs)) return RSAPRNG_E_NULL;
  if (misaligned8(out_u64) || misaligned8(out_f64)) return RSAPRNG_E_ALIGN;
  if (!out_u64 && !out_f64) return RSAPRNG_OK;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return RSAPRNG_E_NO_DEVICE;
  if (dev != pool_device(pool)) return RSAPRNG_E_ARG;
  if (dev < 0 || dev >= kMaxDevices) return RSAPRNG_E_NO_DEVICE;
  Device* d = nullptr;
  int rc;
  // the pool's creation set this device up, so this only looks it up
  if ((rc = device_get(&d))) return rc;
  // two passes or chain-serial (the one-pass form needs look-back words)
  rsaprng_config c = config_for_pool(pool, cfg, kModeGenerate);
  if (c.prefix == kPrefixLookback) {
    c.prefix = kPrefixTwoPass;
    c = config_for_pool(pool, &c, kModeGenerate);
  }
  const u64h T = tile_size(c);
  const u64h chunks_per_tile = T / (64ull * c.per_lane);
  const size_t np = rsaprng_pool_size(pool);

  std::lock_guard<std::mutex> lk(g_mu[dev]);
  PerDevice& pd = g_dev[dev];
  if ((rc = setup(pd))) return rc;
  const int slot = pd.next;
  // the launch that last read this slot's table has finished before it is rewritten
  if (pd.recorded[slot] && hipEventSynchronize(pd.ev[slot]) != hipSuccess) return RSAPRNG_E_HIP;
  Chain* stage = g_stage[dev][slot];

  // Plan straight into the staging table: merge requests that continue each
  // other, then split each range into chains (the steps of plan_chains, in
  // request order).
  u64h nchain = 0, ntiles = 0;
  uint32_t se = 0;
  PlanIn cur;
  bool have = false;
  auto flush = [&](const PlanIn& r) -> int {
    if (r.count == 0) return RSAPRNG_OK;
    Req q;
    u64h nt = 0;
    const int e = plan_one(r, T, ntiles, q, &nt);
    if (e) return e;
    const u64h last = q.k0 + (q.count - 1);
    const u64h chains = (last >> kBlockLog2) - (q.S >> kBlockLog2) + 1;
    if (chains > kMaxChains - nchain) return RSAPRNG_E_TOO_LARGE;
    ntiles += nt;
    plan_emit_chains(q, T, [&](const Chain& ch) { stage[nchain++] = ch; });
    return RSAPRNG_OK;
  };
  for (size_t i = 0; i < nreq; ++i) {
    if (reqs[i].inst >= np) return RSAPRNG_E_ARG;
    const uint32_t e = pool_host(pool, reqs[i].inst).e;
    se = i == 0 ? e : (se == e ? se : 0);
    const PlanIn in{reqs[i].inst, e, reqs[i].k0, reqs[i].count, reqs[i].out_off, 0, 0, 0};
    if (have && plan_merges(cur, in, kModeGenerate)) {
      cur.count += in.count;
      continue;
    }
    if (have && (rc = flush(cur))) return rc;
    cur = in;
    have = true;
  }
  if (have && (rc = flush(cur))) return rc;
  // chain-serial: the lead-in tiles in a pass of their own, the lead-in chains
  // after the output chains in the same table
  LeadIn li;
  li.nout = (uint32_t)nchain;
  if (c.prefix == kPrefixSerial) {
    if ((rc = plan_split_leadin(stage, nchain, kMaxChains, T, &li))) return rc;
    nchain += li.nlead;
  }

  ScratchView v;
  v.ctl = reinterpret_cast<DevCtl*>(pd.ptr);
  v.lb = nullptr;
  v.cstart = reinterpret_cast<ChainStart*>(pd.ptr + kOffCstart);
  v.tiles = reinterpret_cast<uint64_t*>(pd.ptr + kOffTiles);
  v.tiles_cap = ntiles;
  v.chunks_cap = ntiles * chunks_per_tile;
  v.chains_cap = kMaxChains;
  if (ntiles > kTileBytes / 8 || tile_words(v.tiles_cap, v.chunks_cap) > kTileBytes / 8)
    return RSAPRNG_E_TOO_LARGE;
  Chain* dchains = reinterpret_cast<Chain*>(pd.ptr + kOffChains + (size_t)slot * kMaxChains *
                                                                      sizeof(Chain));
  if (nchain && hipMemcpyAsync(dchains, stage, nchain * sizeof(Chain), hipMemcpyHostToDevice,
                               (hipStream_t)stream) != hipSuccess)
    return RSAPRNG_E_HIP;
  rc = enqueue_launch_in(d, v, c, kModeGenerate, pool_dev(pool), nchain ? dchains : nullptr,
                         (uint32_t)nchain, ntiles, out_u64, out_f64, nullptr, 0, nullptr, stream,
                         nullptr, nullptr, se, &li);
  // the slot's table is read by the launch just enqueued (or by the copy
  // already queued if the launch failed): its next writer waits for this event
  if (hipEventRecord(pd.ev[slot], (hipStream_t)stream) != hipSuccess) return rc ? rc : RSAPRNG_E_HIP;
  pd.recorded[slot] = true;
  pd.next = (slot + 1) % kSlots;
  return rc;
}
