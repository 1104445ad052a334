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

// Per-launch scratch owned by the library (one per stream / batch / server).
struct DevCtl {
  uint32_t counter;    // atomic tile queue
  uint32_t epoch;      // tag of this launch's look-back words
  uint32_t err;        // set by a kernel whose bounded wait expired
  uint32_t pad;
};

enum Variant : int { kVariantAuto = 0, kVariantMont = 1, kVariantCrt = 2 };
enum Mode : int { kModeGenerate = 0, kModeConsume = 1 };

struct LaunchArgs {
  const rsaprng_params* inst;
  const Req* req;
  uint32_t nreq;
  uint32_t ntiles;
  uint64_t* out_c;
  double* out_r;
  rsaprng_stats* stats;
  ChainState* state;
  DevCtl* ctl;
  uint64_t* lb;        // 4 tagged words per tile
  const uint64_t* pow2;  // a^(2^i) mod Q, i < 64
  const uint64_t* powv;  // a^(V l) mod Q, l < lanes per tile, for this launch's V
  uint64_t gc;           // a (a - 1)^-1 mod Q: block seed G_b = s0 gc (a^{bB} - 1)
  uint32_t spin_limit;
};

// Host-callable launchers (kernels.hip).
struct KernelShape {
  int variant;   // kVariantMont or kVariantCrt
  int wg;        // 128 or 256
  int v;         // 8 or 16
  int mode;      // kModeGenerate or kModeConsume
  int grid;      // number of work-groups (persistent if < ntiles)
};
int launch_begin(DevCtl* ctl, void* stream);
int launch_tiles(const KernelShape& shape, const LaunchArgs& args, void* stream);
int launch_stats_zero(rsaprng_stats* st, size_t nrec, void* stream);
int launch_stats_finalize(rsaprng_stats* st, size_t nrec, void* stream);
int launch_debug_encrypt(const rsaprng_params& prm, int variant, const uint64_t* m, uint64_t* c,
                         double* r, uint64_t count, void* stream);
int kernel_max_grid(const KernelShape& shape, int* wg_per_cu);

}  // namespace rsaprng
