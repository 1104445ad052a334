// Host-library internals shared by host.cpp and server.cpp.
#pragma once
#include <hip/hip_runtime.h>

#include <vector>

#include "common.h"
#include "plan.h"

namespace rsaprng {

void set_last_error(int e);
bool h_is_prime(u64h n);
u64h h_mulmod(u64h a, u64h b, u64h m);
u64h h_powmod(u64h b, u64h e, u64h m);
u64h h_skip_at(u64h s0, u64h k);
u64h h_block_seed(u64h s0, u64h b);
int h_params(u64h p, u64h q, u64h e, u64h m0, u64h s0, bool check_range, rsaprng_params* out);

struct Device;
int device_get(Device** out);

// Scratch layout in 64-bit words for `cap` tiles and `ccap` wave chunks:
//   tile_chain  uint32 per tile         [0, ceil(cap/2))
//   s_tile      one word per tile       next cap words
//   agg, excl   one word per chunk each next 2 ccap words
inline u64h tile_words(u64h cap, u64h ccap) { return (cap + 1) / 2 + cap + 2 * ccap; }

// Launch scratch (see host.cpp).
struct Scratch {
  struct Slot {
    void* host = nullptr;
    void* dev = nullptr;
    size_t cap = 0;
    hipEvent_t ev = nullptr;
  };
  DevCtl* ctl = nullptr;
  uint64_t* lb = nullptr;        // look-back words, 32 B per tile
  uint64_t* tiles = nullptr;     // tile_chain | s_tile | agg | excl, 32 B per tile
  ChainStart* cstart = nullptr;
  u64h tiles_cap = 0, chunks_cap = 0, chains_cap = 0;
  std::vector<Slot> slots = std::vector<Slot>(4);
  int next_slot = 0;
  ~Scratch();
  int init();
  uint64_t* vec = nullptr;       // vector mode: substream and segment tables
  u64h vec_cap = 0;              // in 64-bit words
  uint32_t* urn2 = nullptr;      // battery: two leading-bit trial bitmaps per work-group slot
  u64h urn2_slots = 0;
  int ensure_tiles(u64h ntiles, u64h nchunks, u64h nchains, void* stream);
  int ensure_vec(u64h words, void* stream);
  int ensure_urn2(u64h slots, void* stream);
  int upload(const void* data, size_t bytes, void* stream, void** dev_out, int* slot_out);
  int mark(int slot, void* stream);
};
int scratch_for_stream(void* stream, Scratch** out);

// The scratch one launch uses: the control block, the look-back words (only
// the one-pass form needs ctl and lb), the tile arrays laid out as tile_words()
// describes for tiles_cap tiles and chunks_cap chunks, and the chain starts
// (one per chain).
struct ScratchView {
  DevCtl* ctl = nullptr;
  uint64_t* lb = nullptr;
  uint64_t* tiles = nullptr;
  ChainStart* cstart = nullptr;
  u64h tiles_cap = 0, chunks_cap = 0, chains_cap = 0;
  uint32_t* urn2 = nullptr;      // battery launches only (kUrn2Words per slot)
  u64h urn2_slots = 0;
};

rsaprng_config resolve_config(const rsaprng_config* cfg);
u64h tile_size(const rsaprng_config& c);
int plan_requests(const PlanIn* in, size_t nreq, const rsaprng_config& c, int mode,
                  std::vector<Req>& out, u64h* ntiles_out);
int plan_chains(const PlanIn* in, size_t nreq, const rsaprng_config& c, int mode,
                std::vector<Chain>& chains, u64h* ntiles_out);
// marks (optional, 5 timing events): recorded before the launch, after chain
// setup, after the prefix pass(es), after the tile kernel and at the end.
int enqueue_launch(Device* d, Scratch* sc, const rsaprng_config& c, int mode,
                   const rsaprng_params* inst, const Chain* chains, uint32_t nchain, u64h ntiles,
                   uint64_t* out_c, double* out_r, rsaprng_stats* stats, size_t nstats,
                   ChainState* state, void* stream, hipEvent_t* marks = nullptr,
                   rsaprng_battery* battery = nullptr, uint32_t shared_e = 0,
                   const LeadIn* li = nullptr);
// The same on scratch the caller provides, sized for the launch (the tile
// arrays for ntiles tiles and their chunks, cstart for nchain chains);
// RSAPRNG_E_ARG if the view is too small.
int enqueue_launch_in(Device* d, const ScratchView& sc, const rsaprng_config& c, int mode,
                      const rsaprng_params* inst, const Chain* chains, uint32_t nchain,
                      u64h ntiles, uint64_t* out_c, double* out_r, rsaprng_stats* stats,
                      size_t nstats, ChainState* state, void* stream, hipEvent_t* marks = nullptr,
                      rsaprng_battery* battery = nullptr, uint32_t shared_e = 0,
                      const LeadIn* li = nullptr);
// Chain-serial generate launches: the lead-in split of plan_split_leadin on a
// planned chain vector (which grows by the lead-in chains); other launches
// are left as planned (li->nlead = 0).
int split_leadin(std::vector<Chain>& chains, const rsaprng_config& c, int mode, LeadIn* li);
// The exponent shared by every request (0 if they differ; dual-exponent
// instances have e = 0): lets a launch take kernels specialised to it.
uint32_t shared_exponent(const PlanIn* in, size_t n);
bool serial16_built(int variant, int mode, uint32_t shared_e, int lanes);
// Parameter generation kernels (k_primes.hip).
int launch_count_primes(uint64_t lo, uint64_t hi, int safe, unsigned long long* count_dev,
                        void* stream);
int launch_next_primes(const uint64_t* x, uint64_t n, int safe, const uint32_t* exps, int nexp,
                       uint64_t span, uint64_t* out, void* stream);

const rsaprng_params* pool_dev(rsaprng_pool_t pool);
const rsaprng_params& pool_host(rsaprng_pool_t pool, size_t i);
int pool_device(rsaprng_pool_t pool);
// The configuration a launch over `pool` uses (CRT for dual-exponent pools).
rsaprng_config config_for_pool(rsaprng_pool_t pool, const rsaprng_config* cfg, int mode);
// Two passes with 16 indices per lane are built for CRT generate launches only;
// other launches of that configuration take four chunks of 8 per wave (the
// same tile).
rsaprng_config fit_mode(rsaprng_config c, int mode);
// Two-pass CRT generate launches with 16 indices per lane: the planned chains
// ordered by exponent class (stable), their tiles renumbered in that order,
// and the class boundaries in li (inst: the pool's host records).  In a launch
// of several classes, a class of fewer than 16384 tiles (the environment
// variable RSAPRNG_CLASS_MIN_TILES overrides it) joins the general class,
// which takes one launch of the per-tile dispatch kernel.  Other launches are
// left as planned (li->nclass = 0).
void group_by_exponent(std::vector<Chain>& chains, const rsaprng_config& c, int mode,
                       const rsaprng_params* inst, LeadIn* li);

}  // namespace rsaprng
