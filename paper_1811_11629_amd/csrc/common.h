// Layouts shared by the host library and the kernels.
#pragma once
#include <stddef.h>
#include <stdint.h>

#include "rsaprng.h"

namespace rsaprng {

constexpr int kBlockLog2 = RSAPRNG_BLOCK_LOG2;
constexpr uint64_t kBlock = 1ull << kBlockLog2;

// One request of a launch: outputs for k in [k0, k0 + count) of instance
// `inst`.  Tiles of the request cover [S, k0 + count) in steps of the tile
// size; S is the scan start (a block start, or a continuation index whose
// chain state is in state[slot]).  Requests are sorted by tile_begin.
struct alignas(16) Req {
  uint64_t k0;
  uint64_t count;
  uint64_t out_off;    // generate: element offset of k0; consume: unused
  uint64_t S;
  uint32_t tile_begin;
  uint32_t inst;
  uint32_t slot;       // chain-state slot (flags) or stats record (consume)
  uint32_t flags;
};
static_assert(sizeof(Req) == 48, "Req layout");

enum ReqFlags : uint32_t {
  kReqContinue = 1u,   // the first tile starts from state[slot] instead of a block seed
  kReqWriteEnd = 2u,   // the tile holding the last index writes state[slot]
};

// Chain state carried between launches (served form): the message just
// before index S and the skip at S.
struct alignas(16) ChainState {
  uint64_t m_prev;     // m_{S-1}
  uint64_t s_at;       // s_S
};

// A chain: the tiles of one request inside one 2^20 block.  Its scan starts at
// S (a block start, or for the first chain of a continued request the index
// whose state is in state[slot]); tiles are T-aligned from S.  The request's
// output range [k0, last] and offset are repeated in every chain.
struct alignas(16) Chain {
  uint64_t S;
  uint64_t k0;
  uint64_t last;
  uint64_t out_off;
  uint32_t inst;
  uint32_t first;      // first tile id
  uint32_t ntiles;
  uint32_t slot;       // chain-state slot or stats record
  uint32_t flags;      // kChainFromState | kChainWriteEnd
  uint32_t pad[3];
};
static_assert(sizeof(Chain) == 64, "Chain layout");

enum ChainFlags : uint32_t {
  kChainFromState = 1u,  // skip and message before S come from state[slot]
  kChainWriteEnd = 2u,   // the tile holding `last` writes state[slot]
  kChainStartGiven = 4u, // the chain's start (skip at S, message before S) is written by
                         // the lead-in pass (k_leadin_state); k_chain_setup leaves it
};

// A chain-serial generate launch whose chains begin with whole tiles before
// their request's first index: those lead-in tiles are walked by the two-pass
// prefix kernels over `nlead` lead-in chains (stored after the `nout` output
// chains, with tiles [0, lead_tiles)), which then hand each output chain its
// start at its first tile with outputs.  nlead = 0: no lead-in pass.
//
// A two-pass CRT generate launch with 16 indices per lane has its chains
// ordered by exponent class: class j holds the tiles [class_end[j-1],
// class_end[j]) (from 0) and exponent class_e[j] (0: any exponent outside the
// unrolled ladders, dual-exponent instances included), and takes the tile
// kernel specialised to it.  nclass = 0: one tile launch.
struct LeadIn {
  uint32_t nout = 0, nlead = 0;
  uint64_t lead_tiles = 0;
  uint32_t nclass = 0;
  uint32_t class_e[7] = {};
  uint64_t class_end[7] = {};
};

// Computed on the device per chain: the skip at S and the message before S,
// and that message's residues mod p and mod q (in (-p, p) and (-q, q)) for the
// CRT kernels.
struct alignas(16) ChainStart {
  uint64_t s_S;
  uint64_t m_base;
  double rp, rq;
};

// Per-launch control words owned by the library (one per stream / batch / server).
struct DevCtl {
  uint32_t counter;    // atomic tile queue (single-pass kernel)
  uint32_t epoch;      // tag of this launch's look-back words
  uint32_t err;        // set by a kernel whose bounded wait expired
  uint32_t pad;
};

enum Variant : int { kVariantAuto = 0, kVariantMont = 1, kVariantCrt = 2 };
enum Mode : int { kModeGenerate = 0, kModeConsume = 1, kModeBattery = 2 };
// How a tile learns the message before it: two passes (tile sums, scan, then
// generate), one pass with a decoupled look-back, or chain-serial (one
// work-group walks a whole chain and carries the prefix from step to step).
enum Prefix : int { kPrefixTwoPass = 0, kPrefixLookback = 1, kPrefixSerial = 2 };

struct LaunchArgs {
  const rsaprng_params* inst;
  const Chain* chain;
  uint32_t nchain;
  uint32_t ntiles;
  uint32_t tile_log2;      // T = 2^tile_log2 indices per tile
  uint32_t chunk_log2;     // a wave's share of a tile: 64 V = 2^chunk_log2 indices
  uint32_t spin_limit;
  uint32_t excl_res;       // two passes, CRT: k_scan leaves the residues of each
                           // chunk's message, mod p in agg and mod q in excl
                           // (binary64 bits), instead of the message in excl
  uint32_t tile0;          // two-pass tile kernel: its tiles are [tile0, ntiles)
  uint32_t* tile_chain;    // per tile: owning chain (k_chain_setup)
  ChainStart* cstart;      // per chain (k_chain_setup)
  uint64_t* s_tile;        // per tile: skip at the tile start (k_sums)
  uint64_t* agg;           // per wave chunk: sum of its skips mod n (k_sums)
  uint64_t* excl;          // per wave chunk: message before the chunk (k_scan; see excl_res)
  uint64_t* lb;            // single pass: 4 tagged words per tile
  uint64_t* out_c;
  double* out_r;
  rsaprng_stats* stats;
  rsaprng_battery* battery;
  ChainState* state;
  DevCtl* ctl;
  const uint64_t* pow2;    // a^(2^i) mod Q, i < 64
  const uint64_t* at;      // a^(j T) mod Q, j < 2^20 / T
  const uint64_t* pl;      // a^((T/64) l) mod Q, l < 64
  const uint64_t* powv;    // a^(V l) mod Q, l < lanes per tile
  uint64_t gc;             // a (a - 1)^-1 mod Q: block seed G_b = s0 gc (a^{bB} - 1)
  uint32_t* urn2;          // battery: per work-group (blockIdx.x) two 2^20-bit bitmaps
                           // of the leading-bit collision trials (kUrn2Words words)
};

// Leading-bit collision trials of the battery (rsaprng.h): balls of 20
// indices, 2^14 balls per trial, three trials per 2^20 block; a work-group's
// two bitmaps (by trial parity) in device memory.
constexpr uint64_t kMsbBall = 20;
constexpr uint64_t kMsbTrial = kMsbBall << 14;
constexpr int kMsbTrials = 3;
constexpr uint32_t kUrn2Words = 2u * ((1u << 20) / 32);

// Vector mode (k_vector.hip): one launch over vector calls [t_lo, t_hi] of one
// instance.  Lane j stands for substream g = (g_lo + j) mod mv; segment i of
// the domain holds indices [(sig_a + i) W, (sig_a + i + 1) W), W = 2^w with
// 6 <= w <= 19; groups of 2^glog2 consecutive segments lie inside one block.  The output of (k, g)
// goes to out[(k - t_lo) mv + g - g_lo] when that lies in [0, count).
struct VecArgs {
  rsaprng_params P;
  const uint64_t* pow2;    // a^(2^i) mod Q
  uint64_t gc;             // a (a - 1)^-1 mod Q
  uint64_t mv;             // M_v
  uint64_t J;              // floor((Q - 1) / M_v)
  uint64_t g_lo;           // substream of the first output
  uint64_t t_lo, t_hi;     // first and last vector call (substream index k)
  uint64_t count;          // outputs of the launch
  uint64_t sig_a;          // first segment of the domain (a block start)
  uint32_t ng;             // substreams in play
  uint32_t nseg, ngrp, nblk;
  uint32_t osig, noseg;    // segments holding outputs: [osig, osig + noseg)
  uint32_t w, glog2;
  uint64_t* va;            // [ng]        s0 a^(g J) mod Q
  uint64_t* vb;            // [nseg]      a^((sig_a + i) W) mod Q
  uint64_t* vagg;          // [nseg][ng]  segment sums, then in-group prefixes
  uint64_t* vgrp;          // [ngrp][ng]  group totals, then message before each group
  uint64_t* out_c;
  double* out_r;
};
int launch_vector(const VecArgs& args, int variant, void* stream);

// Host-callable launchers (kernels.hip).
struct KernelShape {
  int variant;   // kVariantMont or kVariantCrt
  int wg;        // 256 or 512
  int v;         // 8 or 16
  int mode;      // kModeGenerate or kModeConsume
  int prefix;    // kPrefixTwoPass, kPrefixLookback or kPrefixSerial
  int r;         // two passes: consecutive wave chunks per wave (tile = wg v r)
  int grid;      // number of work-groups (they loop if fewer than tiles)
  uint32_t e;    // the exponent of every instance of the launch, or 0 if they differ
};
int launch_begin(DevCtl* ctl, void* stream);
int launch_chain_setup(const LaunchArgs& args, void* stream);
int launch_sums(const LaunchArgs& args, void* stream);
int launch_scan(const LaunchArgs& args, void* stream);
int launch_tiles(const KernelShape& shape, const LaunchArgs& args, void* stream);
int launch_battery_zero(rsaprng_battery* rec, uint64_t outputs, void* stream);
// slots: the work-group slots of args.urn2 (the grid is capped to them)
int launch_battery_values(const LaunchArgs& args, const double* r, uint64_t count, uint32_t slots,
                          void* stream);
int launch_stats_zero(rsaprng_stats* st, size_t nrec, void* stream);
// For each lead-in chain l of `lead` (its prefix arrays filled by k_sums and
// k_scan): out[slot of l] = the skip at the first index after its tiles and
// the message before it.
int launch_leadin_state(const LaunchArgs& lead, ChainStart* out, void* stream);
int launch_stats_finalize(rsaprng_stats* st, size_t nrec, void* stream);
int launch_debug_encrypt(const rsaprng_params& prm, int variant, const uint64_t* m, uint64_t* c,
                         double* r, uint64_t count, void* stream);
int kernel_max_grid(const KernelShape& shape, int* wg_per_cu);
int launch_checksum(const uint64_t* p, uint64_t n, uint64_t* out_dev, void* stream);
// p[i] = v for i < n.
int launch_fill(uint64_t* p, uint64_t n, uint64_t v, void* stream);
// Throughput probes (k_probe.hip).
int probe_grid(int ncu);
uint64_t probe_threads(int ncu);
uint64_t probe_ops_per_thread(uint64_t iters);
int launch_probe(int kind, int ncu, uint64_t n, uint64_t* out_u64, double* out_f64, void* stream);

}  // namespace rsaprng
