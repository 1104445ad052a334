// Host-only driver of the whole host library (host.cpp, server.cpp,
// noalloc.hip) over the checking runtime of fakehip.cpp, for sanitizer builds.
//
// The kernel launchers are replaced here by functions that queue, on the
// launch's stream, a check of every range the real kernel would touch against
// the live device allocations, and the writes the real kernel makes in a form
// the harness can check: every generated output is a tag of (instance, index),
// chain-end states are tags of the last index, statistics records count their
// outputs, and the prefix arrays carry the owning chain.  The library then runs
// the request sets of the workloads (uneven batched requests with k0 below
// 2^40, consume records, served requests arriving in waves) through every
// entry point; each output must hold the tag of its own (instance, index),
// each gap between requests its sentinel, and the device objects created by a
// batch, a server or an autotuner run must be gone after it is destroyed.
// Prints "ok <summary>" or the first violation (exit status 1; the runtime's
// own violations exit with status 3).
#include <hip/hip_runtime.h>

#include <array>
#include <cinttypes>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>
#include <string>
#include <vector>

#include "common.h"

using namespace rsaprng;

#define CHECK(c, ...)                         \
  do {                                        \
    if (!(c)) {                               \
      std::printf("violation: " __VA_ARGS__); \
      std::printf(" (line %d)\n", __LINE__);  \
      std::fflush(stdout);                    \
      std::exit(1);                           \
    }                                         \
  } while (0)

namespace {

constexpr uint64_t kSentinel = 0x5A5A5A5A5A5A5A5Aull;

uint64_t mix(uint64_t z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
uint64_t tag_c(uint32_t inst, uint64_t k) { return mix(((uint64_t)inst << 40) ^ mix(k)); }
uint64_t tag_r(uint32_t inst, uint64_t k) { return ~tag_c(inst, k); }
uint64_t tag_state(uint32_t inst, uint64_t k) { return mix(tag_c(inst, k) + 17); }
uint64_t marker(uint32_t c) { return 0xC4A1000000000000ull | c; }

template <class T>
T rd(const T* p, const char* what) {
  fakehip::need_device(p, sizeof(T), what);
  return *p;
}
template <class T>
void wr(T* p, const T& v, const char* what) {
  fakehip::need_device(p, sizeof(T), what);
  *p = v;
}

int enq(void* stream, const char* what, std::function<void()> f) {
  fakehip::enqueue((hipStream_t)stream, what, std::move(f));
  return RSAPRNG_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// the kernel launchers
// ---------------------------------------------------------------------------
namespace rsaprng {

bool serial16_built(int variant, int mode, uint32_t shared_e, int lanes);  // host.cpp

int launch_begin(DevCtl* ctl, void* stream) {
  return enq(stream, "k_begin", [=] {
    DevCtl c = rd(ctl, "k_begin ctl");
    c.counter = 0;
    c.epoch = c.epoch + 1 ? c.epoch + 1 : 1;
    wr(ctl, c, "k_begin ctl");
  });
}

static Chain chain_at(const LaunchArgs& a, uint32_t c, const char* what) {
  const Chain C = rd(a.chain + c, what);
  (void)rd(a.inst + C.inst, what);  // the instance record is read
  return C;
}

int launch_chain_setup(const LaunchArgs& a, void* stream) {
  if (!a.nchain) return RSAPRNG_OK;
  return enq(stream, "k_chain_setup", [a] {
    const uint64_t T = 1ull << a.tile_log2;
    for (uint32_t c = 0; c < a.nchain; ++c) {
      const Chain C = chain_at(a, c, "k_chain_setup chain");
      CHECK((uint64_t)C.first + C.ntiles <= a.ntiles, "chain %u tiles [%u, +%u) beyond %u", c,
            C.first, C.ntiles, a.ntiles);
      CHECK(C.S % T == 0, "chain %u start %" PRIu64 " not tile-aligned", c, C.S);
      if (C.flags & kChainFromState) {
        const ChainState st = rd(a.state + C.slot, "k_chain_setup state");
        CHECK(C.S > 0 && st.m_prev == tag_state(C.inst, C.S - 1),
              "chain %u continues from a state that is not the one before index %" PRIu64, c, C.S);
      }
      for (uint32_t i = 0; i < C.ntiles; ++i) wr(a.tile_chain + C.first + i, c, "tile_chain");
      if (C.flags & kChainStartGiven) {
        // the lead-in pass writes it; mark it unset until then
        wr(a.cstart + c, ChainStart{0, 0}, "cstart (given later)");
      } else {
        wr(a.cstart + c, ChainStart{marker(c), marker(c)}, "cstart");
      }
    }
  });
}

int launch_sums(const LaunchArgs& a, void* stream) {
  if (!a.ntiles) return RSAPRNG_OK;
  return enq(stream, "k_sums", [a] {
    const uint64_t ch = 1ull << (a.tile_log2 - a.chunk_log2);
    for (uint32_t t = 0; t < a.ntiles; ++t) {
      const uint32_t c = rd(a.tile_chain + t, "k_sums tile_chain");
      CHECK(c < a.nchain, "tile %u owned by chain %u of %u", t, c, a.nchain);
      CHECK(rd(a.cstart + c, "k_sums cstart").s_S == marker(c), "k_sums: chain start unset");
      wr(a.s_tile + t, marker(c), "s_tile");
      for (uint64_t j = 0; j < ch; ++j) wr(a.agg + t * ch + j, marker(c), "agg");
    }
  });
}

int launch_scan(const LaunchArgs& a, void* stream) {
  if (!a.nchain) return RSAPRNG_OK;
  return enq(stream, "k_scan", [a] {
    const uint64_t ch = 1ull << (a.tile_log2 - a.chunk_log2);
    for (uint32_t c = 0; c < a.nchain; ++c) {
      const Chain C = chain_at(a, c, "k_scan chain");
      for (uint64_t q = (uint64_t)C.first * ch; q < ((uint64_t)C.first + C.ntiles) * ch; ++q) {
        CHECK(rd(a.agg + q, "k_scan agg") == marker(c), "chunk %" PRIu64 " sum not of chain %u",
              q, c);
        wr(a.excl + q, marker(c), "excl");
      }
    }
  });
}

int launch_leadin_state(const LaunchArgs& a, ChainStart* out, void* stream) {
  if (!a.nchain) return RSAPRNG_OK;
  return enq(stream, "k_leadin_state", [a, out] {
    const uint64_t ch = 1ull << (a.tile_log2 - a.chunk_log2);
    const uint64_t T = 1ull << a.tile_log2;
    for (uint32_t l = 0; l < a.nchain; ++l) {
      const Chain L = chain_at(a, l, "k_leadin_state chain");
      const uint64_t q = ((uint64_t)L.first + L.ntiles) * ch - 1;
      CHECK(L.k0 == L.S && L.last == L.S + L.ntiles * T - 1 && L.ntiles > 0,
            "lead-in chain %u malformed", l);
      CHECK(rd(a.excl + q, "lead excl") == marker(l) && rd(a.agg + q, "lead agg") == marker(l),
            "lead-in chain %u: prefix of its last chunk unset", l);
      (void)rd(a.cstart + l, "lead cstart");
      (void)rd(a.at + L.ntiles, "a^(T ntiles)");
      wr(out + L.slot, ChainStart{marker(L.slot), marker(L.slot)}, "output chain start");
    }
  });
}

int launch_tiles(const KernelShape& s, const LaunchArgs& a, void* stream) {
  if (s.grid < 1) return RSAPRNG_E_ARG;
  return enq(stream, "tile kernel", [s, a] {
    const uint64_t T = 1ull << a.tile_log2;
    const uint64_t ch = 1ull << (a.tile_log2 - a.chunk_log2);
    CHECK(T == (uint64_t)s.wg * s.v * (s.prefix == kPrefixLookback ? 1 : s.r),
          "tile size %" PRIu64 " does not match the kernel shape", T);
    // chain-serial kernels with 16 indices per lane exist only specialised to
    // one exponent; the lane-offset table must be the one for 16
    if (s.prefix == kPrefixSerial && s.v == 16)
      CHECK(s.r == 1 && serial16_built(s.variant, s.mode, s.e, s.wg),
            "no chain-serial kernel (%d, 16, %d) for variant %d mode %d e = %u", s.wg, s.r,
            s.variant, s.mode, s.e);
    if (s.prefix == kPrefixSerial) CHECK(s.v == 8 || s.v == 16, "indices per lane %d", s.v);
    // two passes with 16 indices per lane: CRT generate only; the launch may
    // cover one exponent class's tiles [tile0, ntiles)
    if (s.prefix == kPrefixTwoPass && s.v == 16)
      CHECK(s.variant == kVariantCrt && s.mode == kModeGenerate && s.r == 2,
            "no two-pass kernel (%d, 16, %d) for variant %d mode %d", s.wg, s.r, s.variant, s.mode);
    CHECK(a.tile0 < a.ntiles, "empty tile range [%u, %u)", a.tile0, a.ntiles);
    CHECK(a.tile0 == 0 || (s.prefix == kPrefixTwoPass && s.v == 16),
          "a tile range from %u outside the exponent classes", a.tile0);
    if (s.prefix == kPrefixLookback) {
      (void)rd(a.ctl, "look-back ctl");
      fakehip::need_device(a.lb, (size_t)a.ntiles * 32, "look-back words");
    }
    for (uint32_t c = 0; c < a.nchain; ++c) {
      const Chain C = chain_at(a, c, "tile chain");
      // chains outside this launch's tile range belong to another class's launch
      if (C.first + C.ntiles <= a.tile0 || C.first >= a.ntiles) continue;
      CHECK(C.first >= a.tile0 && C.first + C.ntiles <= a.ntiles,
            "chain %u tiles [%u, +%u) straddle the launch's range [%u, %u)", c, C.first, C.ntiles,
            a.tile0, a.ntiles);
      const rsaprng_params P = rd(a.inst + C.inst, "tile instance");
      if (s.e) CHECK(P.e == s.e, "launch specialised to e = %u holds e = %u", s.e, P.e);
      for (uint32_t t = C.first; t < C.first + C.ntiles; ++t) {
        CHECK(rd(a.tile_chain + t, "tile_chain") == c, "tile %u not of chain %u", t, c);
        if (s.prefix == kPrefixTwoPass) {
          (void)rd(a.s_tile + t, "s_tile");
          for (uint64_t j = 0; j < ch; ++j)
            CHECK(rd(a.excl + (uint64_t)t * ch + j, "excl") == marker(c),
                  "tile %u chunk prefix not of chain %u", t, c);
        }
      }
      CHECK(rd(a.cstart + c, "cstart").m_base == marker(c), "chain %u start unset", c);
      const uint64_t bs = C.S & ~(kBlock - 1), be = bs + (kBlock - 1);
      const unsigned __int128 tend = (unsigned __int128)C.S + (unsigned __int128)C.ntiles * T;
      CHECK(tend <= (unsigned __int128)be + 1, "chain %u tiles cross the block end", c);
      CHECK(C.k0 <= C.last, "chain %u: empty request", c);
      const uint64_t lo = C.S > C.k0 ? C.S : C.k0, hi = C.last < be ? C.last : be;
      if (lo <= hi) CHECK((unsigned __int128)hi < tend, "chain %u: tiles miss index %" PRIu64, c, hi);
      for (uint64_t k = lo; lo <= hi && k <= hi; ++k) {
        if (s.mode == kModeGenerate) {
          const uint64_t j = C.out_off + (k - C.k0);
          if (a.out_c) wr(a.out_c + j, tag_c(C.inst, k), "out_c");
          if (a.out_r) wr(reinterpret_cast<uint64_t*>(a.out_r) + j, tag_r(C.inst, k), "out_r");
        }
        if (k == hi) break;
      }
      if (s.mode == kModeConsume && lo <= hi) {
        rsaprng_stats* st = a.stats + C.slot;
        fakehip::need_device(st, sizeof(*st), "stats record");
        st->count += hi - lo + 1;
      }
      if (s.mode == kModeBattery) {
        fakehip::need_device(a.battery, sizeof(rsaprng_battery), "battery record");
        // the leading-bit bitmaps of the work-group slots the grid uses
        fakehip::need_device(a.urn2, (size_t)s.grid * kUrn2Words * sizeof(uint32_t), "battery bitmaps");
      }
      if ((C.flags & kChainWriteEnd) && C.last <= be)
        wr(a.state + C.slot, ChainState{tag_state(C.inst, C.last), 0}, "chain-end state");
    }
  });
}

int launch_battery_zero(rsaprng_battery* rec, uint64_t outputs, void* stream) {
  return enq(stream, "k_battery_zero", [=] {
    fakehip::need_device(rec, sizeof(*rec), "battery record");
    std::memset(rec, 0, sizeof(*rec));
    rec->outputs = outputs;
  });
}

int launch_battery_values(const LaunchArgs& a, const double* r, uint64_t count, uint32_t slots,
                          void* stream) {
  if (count && (!a.urn2 || slots == 0)) return RSAPRNG_E_ARG;
  return enq(stream, "k_battery_values", [=] {
    fakehip::need_device(r, count * 8, "battery values");
    fakehip::need_device(a.battery, sizeof(rsaprng_battery), "battery record");
    if (count) fakehip::need_device(a.urn2, (size_t)slots * kUrn2Words * sizeof(uint32_t), "battery bitmaps");
  });
}

int launch_stats_zero(rsaprng_stats* st, size_t nrec, void* stream) {
  return enq(stream, "k_stats_zero", [=] {
    fakehip::need_device(st, nrec * sizeof(rsaprng_stats), "stats records");
    std::memset(st, 0, nrec * sizeof(rsaprng_stats));
  });
}

int launch_stats_finalize(rsaprng_stats* st, size_t nrec, void* stream) {
  return enq(stream, "k_stats_finalize", [=] {
    fakehip::need_device(st, nrec * sizeof(rsaprng_stats), "stats records");
  });
}

int launch_debug_encrypt(const rsaprng_params&, int, const uint64_t* m, uint64_t* c, double* r,
                         uint64_t count, void* stream) {
  return enq(stream, "k_debug_encrypt", [=] {
    fakehip::need_device(m, count * 8, "debug m");
    if (c) fakehip::need_device(c, count * 8, "debug c");
    if (r) fakehip::need_device(r, count * 8, "debug r");
  });
}

int kernel_max_grid(const KernelShape&, int* wg_per_cu) {
  *wg_per_cu = 2;
  return RSAPRNG_OK;
}

int launch_checksum(const uint64_t* p, uint64_t n, uint64_t* out_dev, void* stream) {
  return enq(stream, "k_checksum", [=] {
    fakehip::need_device(p, n * 8, "checksum input");
    uint64_t h = 1469598103934665603ull;
    for (uint64_t i = 0; i < n; ++i) h = (h ^ p[i]) * 1099511628211ull;
    wr(out_dev, h, "checksum out");
  });
}

int launch_fill(uint64_t* p, uint64_t n, uint64_t v, void* stream) {
  return enq(stream, "k_fill", [=] {
    fakehip::need_device(p, n * 8, "fill");
    for (uint64_t i = 0; i < n; ++i) p[i] = v;
  });
}

int probe_grid(int ncu) { return ncu * 8; }
uint64_t probe_threads(int ncu) { return (uint64_t)probe_grid(ncu) * 256; }
uint64_t probe_ops_per_thread(uint64_t iters) { return iters * 32; }

int launch_probe(int kind, int ncu, uint64_t n, uint64_t* out_u64, double* out_f64,
                 void* stream) {
  return enq(stream, "k_probe", [=] {
    if (kind >= RSAPRNG_PROBE_STORE_TILE) {
      fakehip::need_device(out_u64, n * 8, "probe out");
      fakehip::need_device(out_f64, n * 8, "probe out");
    } else {
      fakehip::need_device(out_u64, probe_threads(ncu) * 8, "probe sink");
    }
  });
}

int launch_vector(const VecArgs& v, int, void* stream) {
  return enq(stream, "k_vector", [v] {
    fakehip::need_device(v.va, (size_t)v.ng * 8, "vector va");
    fakehip::need_device(v.vb, (size_t)v.nseg * 8, "vector vb");
    fakehip::need_device(v.vagg, (size_t)v.nseg * v.ng * 8, "vector vagg");
    fakehip::need_device(v.vgrp, (size_t)v.ngrp * v.ng * 8, "vector vgrp");
    if (v.out_c) fakehip::need_device(v.out_c, v.count * 8, "vector out_c");
    if (v.out_r) fakehip::need_device(v.out_r, v.count * 8, "vector out_r");
  });
}

int launch_count_primes(uint64_t, uint64_t, int, unsigned long long* count_dev, void* stream) {
  return enq(stream, "k_count_primes", [=] { wr(count_dev, 0ull, "prime count"); });
}

int launch_next_primes(const uint64_t* x, uint64_t n, int, const uint32_t* exps, int nexp,
                       uint64_t, uint64_t* out, void* stream) {
  std::vector<uint32_t> ex(exps, exps + nexp);  // read when enqueued, as kernel arguments are
  return enq(stream, "k_next_primes", [=] {
    fakehip::need_device(x, n * 8, "next_primes x");
    fakehip::need_device(out, n * 8, "next_primes out");
    (void)ex;
  });
}

}  // namespace rsaprng

// ---------------------------------------------------------------------------
// the driver
// ---------------------------------------------------------------------------
namespace {

std::mt19937_64 rng(20261203);

struct HReq {
  uint32_t inst;
  uint64_t k0, count, off;
};

uint64_t next_prime(uint64_t x) {
  while (!rsaprng_is_prime(x)) ++x;
  return x;
}

rsaprng_pool_t make_pool(size_t n, std::vector<uint32_t>* es, bool one_e = false) {
  static const uint64_t kE[] = {3, 5, 7, 17, 257, 65537};
  std::vector<uint64_t> p(n), q(n), e(n), seed(n);
  for (size_t i = 0; i < n; ++i) {
    for (;;) {
      p[i] = next_prime((1ull << 31) + (rng() >> 33));
      q[i] = next_prime((1ull << 31) + (rng() >> 33));
      e[i] = one_e ? 3 : kE[rng() % 6];
      rsaprng_params prm;
      if (p[i] < (1ull << 32) && q[i] < (1ull << 32) &&
          rsaprng_params_init(p[i], q[i], e[i], 1, 1, &prm) == RSAPRNG_OK)
        break;
    }
    seed[i] = rng();
  }
  size_t bad = 0;
  rsaprng_pool_t pool = rsaprng_pool_create(n, p.data(), q.data(), e.data(), seed.data(), nullptr,
                                            &bad);
  CHECK(pool, "pool_create failed at %zu (%d)", bad, rsaprng_last_error());
  if (es) es->assign(e.begin(), e.end());
  return pool;
}

// Uneven requests: lengths log-uniform in [2^lo, 2^hi), k0 < 2^40 (some near
// the top of the index range, some continuing the previous request), packed
// back to back with a one-element gap after every third.
std::vector<HReq> uneven(size_t n, uint32_t ninst, int lo, int hi, uint64_t* total) {
  std::vector<HReq> v;
  uint64_t off = 0;
  for (size_t j = 0; j < n; ++j) {
    HReq r;
    r.inst = (uint32_t)(rng() % ninst);
    const double u = (double)(rng() >> 11) / 9007199254740992.0;
    r.count = (uint64_t)std::exp2(lo + (hi - lo) * u);
    r.k0 = rng() >> 24;
    if (j % 17 == 5) r.k0 = 0ull - r.count;  // ends at index 2^64 - 1
    if (j % 13 == 7 && !v.empty()) {        // continues the previous request
      r.inst = v.back().inst;
      r.k0 = v.back().k0 + v.back().count;
      if (r.k0 + r.count < r.k0) r.k0 = 0;
    }
    r.off = off;
    off += r.count + (j % 3 == 0);
    v.push_back(r);
  }
  *total = off;
  return v;
}

std::vector<rsaprng_pool_req> pool_reqs(const std::vector<HReq>& v, bool consume = false) {
  std::vector<rsaprng_pool_req> out;
  for (size_t i = 0; i < v.size(); ++i)
    out.push_back(rsaprng_pool_req{v[i].inst, 0, v[i].k0, v[i].count, consume ? i : v[i].off});
  return out;
}

struct Outputs {
  uint64_t* c = nullptr;
  double* r = nullptr;
  uint64_t n = 0;
  explicit Outputs(uint64_t n_) : n(n_) {
    CHECK(hipMalloc(&c, n * 8 + 8) == hipSuccess && hipMalloc(&r, n * 8 + 8) == hipSuccess,
          "hipMalloc");
    clear();
  }
  ~Outputs() {
    (void)hipFree(c);
    (void)hipFree(r);
  }
  void clear() {
    std::vector<uint64_t> s(n, kSentinel);
    CHECK(hipMemcpy(c, s.data(), n * 8, hipMemcpyHostToDevice) == hipSuccess, "clear");
    CHECK(hipMemcpy(r, s.data(), n * 8, hipMemcpyHostToDevice) == hipSuccess, "clear");
  }
  void verify(const std::vector<HReq>& v, const char* what, uint64_t gap = kSentinel) {
    fakehip::drain();
    std::vector<uint64_t> hc(n), hr(n);
    CHECK(hipMemcpy(hc.data(), c, n * 8, hipMemcpyDeviceToHost) == hipSuccess, "read");
    CHECK(hipMemcpy(hr.data(), r, n * 8, hipMemcpyDeviceToHost) == hipSuccess, "read");
    std::vector<char> w(n, 0);
    for (const HReq& q : v)
      for (uint64_t j = 0; j < q.count; ++j) {
        const uint64_t o = q.off + j;
        CHECK(hc[o] == tag_c(q.inst, q.k0 + j) && hr[o] == tag_r(q.inst, q.k0 + j),
              "%s: output %" PRIu64 " (inst %u, k %" PRIu64 ") wrong", what, o, q.inst, q.k0 + j);
        w[o] = 1;
      }
    for (uint64_t o = 0; o < n; ++o)
      CHECK(w[o] || (hc[o] == gap && hr[o] == gap), "%s: gap %" PRIu64 " written", what, o);
  }
};

rsaprng_config cfg_of(int variant, int prefix, int lanes, int r, int persistent, int per = 8) {
  rsaprng_config c;
  std::memset(&c, 0, sizeof(c));
  c.variant = variant;
  c.prefix = prefix;
  c.lanes_per_tile = lanes;
  c.per_lane = per;
  c.chunks_per_wave = r;
  c.persistent = persistent;
  c.order = persistent;
  return c;
}

// (prefix, lanes, chunks per wave, indices per lane)
const int kShapes[][4] = {{0, 256, 1, 8}, {0, 256, 2, 8}, {0, 256, 4, 8}, {0, 512, 2, 8}, {0, 256, 2, 16},
                          {1, 256, 1, 8}, {1, 512, 1, 8}, {1, 256, 1, 16}, {2, 256, 2, 8},
                          {2, 256, 4, 8}, {2, 512, 2, 8}, {2, 256, 1, 16}, {2, 512, 1, 16}};

hipStream_t new_stream() {
  hipStream_t s;
  CHECK(hipStreamCreateWithFlags(&s, hipStreamNonBlocking) == hipSuccess, "stream");
  return s;
}

}  // namespace

int main(int argc, char** argv) {
  const char* cache = argc > 1 ? argv[1] : "/tmp/rsaprng_harness_tune.jsonl";
  // every exponent class of a grouped two-pass launch takes a launch of its
  // own, however few its tiles (the harness's launches are small)
  setenv("RSAPRNG_CLASS_MIN_TILES", "0", 1);
  std::remove(cache);
  std::vector<uint32_t> es;
  rsaprng_pool_t pool = make_pool(300, &es);
  rsaprng_pool_t pool3 = make_pool(40, nullptr, true);
  hipStream_t st = new_stream();
  long checked = 0;

  // 1. pool_generate over uneven requests, every shape, both variants, persistent or not
  {
    uint64_t total;
    auto v = uneven(400, 300, 4, 13, &total);
    auto pr = pool_reqs(v);
    Outputs o(total);
    for (int var : {1, 2})
      for (const auto& sh : kShapes)
        for (int pers : {0, 1}) {
          o.clear();
          rsaprng_config c = cfg_of(var, sh[0], sh[1], sh[2], pers, sh[3]);
          CHECK(rsaprng_pool_generate(pool, pr.data(), pr.size(), o.c, o.r, &c, st) == RSAPRNG_OK,
                "pool_generate");
          o.verify(v, "pool_generate");
          checked += (long)total;
        }
    // a launch whose requests all have e = 3 (the specialised kernels)
    auto v3 = uneven(60, 40, 4, 14, &total);
    auto pr3 = pool_reqs(v3);
    Outputs o3(total);
    for (const auto& sh : {std::array<int, 3>{512, 2, 8}, std::array<int, 3>{256, 1, 16},
                           std::array<int, 3>{512, 1, 16}}) {
      o3.clear();
      rsaprng_config c = cfg_of(2, 2, sh[0], sh[1], 0, sh[2]);
      CHECK(rsaprng_pool_generate(pool3, pr3.data(), pr3.size(), o3.c, o3.r, &c, st) ==
                RSAPRNG_OK,
            "pool_generate e = 3");
      o3.verify(v3, "pool_generate e = 3");
    }
    CHECK(rsaprng_check_device_error(st) == RSAPRNG_OK, "device error");
  }

  // 2. the no-allocation entry point: two calls in a row (the second smaller), then its limits
  {
    uint64_t t1, t2;
    auto v1 = uneven(300, 300, 4, 14, &t1);
    auto v2 = uneven(20, 300, 2, 9, &t2);
    auto p1 = pool_reqs(v1), p2 = pool_reqs(v2);
    Outputs o1(t1), o2(t2);
    for (const auto& sh : kShapes) {
      o1.clear();
      o2.clear();
      rsaprng_config c = cfg_of(2, sh[0], sh[1], sh[2], 0, sh[3]);
      CHECK(rsaprng_pool_generate_noalloc(pool, p1.data(), p1.size(), o1.c, o1.r, &c, st) ==
                RSAPRNG_OK,
            "noalloc call 1");
      CHECK(rsaprng_pool_generate_noalloc(pool, p2.data(), p2.size(), o2.c, o2.r, &c, st) ==
                RSAPRNG_OK,
            "noalloc call 2");
      // a third call on another stream reuses the first upload slot: it waits
      hipStream_t s2 = new_stream();
      CHECK(rsaprng_pool_generate_noalloc(pool, p2.data(), p2.size(), o2.c, o2.r, &c, s2) ==
                RSAPRNG_OK,
            "noalloc call 3");
      o1.verify(v1, "noalloc call 1");
      o2.verify(v2, "noalloc call 2");
      CHECK(hipStreamDestroy(s2) == hipSuccess, "stream");
      checked += (long)(t1 + t2);
    }
    const size_t dev_before = fakehip::live_device_allocations();
    Outputs small(4);
    std::vector<rsaprng_pool_req> many;
    for (uint32_t j = 0; j <= RSAPRNG_NOALLOC_MAX_CHAINS; ++j)
      many.push_back(rsaprng_pool_req{j % 300, 0, (uint64_t)j << 20, 1, 0});
    CHECK(rsaprng_pool_generate_noalloc(pool, many.data(), many.size(), small.c, small.r, nullptr,
                                        st) == RSAPRNG_E_TOO_LARGE,
          "too many chains");
    // beyond the scratch for every shape (16 indices per lane halve the chunk
    // records: about 1.7e9 outputs fit them)
    for (uint64_t cnt : {1ull << 31, 1ull << 32}) {
      rsaprng_pool_req big{0, 0, 0, cnt, 0};
      for (const auto& sh : kShapes) {
        rsaprng_config c = cfg_of(2, sh[0], sh[1], sh[2], 0, sh[3]);
        CHECK(rsaprng_pool_generate_noalloc(pool, &big, 1, small.c, small.r, &c, st) ==
                  RSAPRNG_E_TOO_LARGE,
              "tile arrays beyond the scratch (count %" PRIu64 ")", cnt);
      }
    }
    rsaprng_pool_req wrap{0, 0, 2, ~0ull, 0};
    CHECK(rsaprng_pool_generate_noalloc(pool, &wrap, 1, small.c, small.r, nullptr, st) ==
              RSAPRNG_E_RANGE,
          "k0 + count > 2^64");
    rsaprng_pool_req badi{300, 0, 0, 10, 0};
    CHECK(rsaprng_pool_generate_noalloc(pool, &badi, 1, small.c, small.r, nullptr, st) ==
              RSAPRNG_E_ARG,
          "instance out of range");
    std::vector<HReq> none;
    small.verify(none, "after the failed calls");  // nothing was written
    rsaprng_pool_req one{7, 0, 5, 4, 0};
    CHECK(rsaprng_pool_generate_noalloc(pool, &one, 1, small.c, small.r, nullptr, st) ==
              RSAPRNG_OK,
          "noalloc after errors");
    small.verify({HReq{7, 5, 4, 0}}, "noalloc after errors");
    CHECK(fakehip::live_device_allocations() == dev_before + 2, "noalloc allocated device memory");
  }

  // 3. consume over per-request records; the same through a prepared batch
  {
    uint64_t total;
    auto v = uneven(64, 300, 6, 14, &total);
    auto pr = pool_reqs(v, true);
    rsaprng_stats* stats;
    CHECK(hipMalloc(&stats, v.size() * sizeof(rsaprng_stats)) == hipSuccess, "stats");
    auto check_stats = [&](const char* what) {
      fakehip::drain();
      std::vector<rsaprng_stats> h(v.size());
      CHECK(hipMemcpy(h.data(), stats, h.size() * sizeof(rsaprng_stats), hipMemcpyDeviceToHost) ==
                hipSuccess,
            "read stats");
      for (size_t i = 0; i < v.size(); ++i)
        CHECK(h[i].count == v[i].count, "%s: record %zu counts %" PRIu64 " of %" PRIu64, what, i,
              h[i].count, v[i].count);
    };
    for (const auto& sh : kShapes) {
      rsaprng_config c = cfg_of(2, sh[0], sh[1], sh[2], 1, sh[3]);
      CHECK(rsaprng_pool_consume(pool, pr.data(), pr.size(), stats, &c, st) == RSAPRNG_OK,
            "pool_consume");
      check_stats("pool_consume");
      rsaprng_batch_t b;
      CHECK(rsaprng_batch_create(pool, pr.data(), pr.size(), 1, nullptr, nullptr, stats, &c, st,
                                 &b) == RSAPRNG_OK,
            "batch_create consume");
      for (int i = 0; i < 3; ++i) CHECK(rsaprng_batch_run(b, st) == RSAPRNG_OK, "batch_run");
      check_stats("consume batch");
      rsaprng_batch_destroy(b);
    }
    CHECK(hipFree(stats) == hipSuccess, "free stats");
  }

  // 4. prepared batches (graph and timed eager form) over uneven generate requests;
  //    nothing they created outlives them
  {
    uint64_t total;
    auto v = uneven(300, 300, 4, 13, &total);
    auto pr = pool_reqs(v);
    Outputs o(total);
    const size_t d0 = fakehip::live_device_allocations(), s0 = fakehip::live_streams(),
                 e0 = fakehip::live_events();
    for (const auto& sh : kShapes)
      for (int pers : {0, 1}) {
        rsaprng_config c = cfg_of(2, sh[0], sh[1], sh[2], pers, sh[3]);
        rsaprng_batch_t b;
        CHECK(rsaprng_batch_create(pool, pr.data(), pr.size(), 0, o.c, o.r, nullptr, &c, st, &b) ==
                  RSAPRNG_OK,
              "batch_create");
        for (int rep = 0; rep < 2; ++rep) {
          o.clear();
          CHECK(rsaprng_batch_run(b, st) == RSAPRNG_OK, "batch_run");
          o.verify(v, "graph replay");
        }
        o.clear();
        for (int rep = 0; rep < 3; ++rep)
          CHECK(rsaprng_batch_run_timed(b, st) == RSAPRNG_OK, "batch_run_timed");
        double ms[4];
        int runs = 0;
        CHECK(rsaprng_batch_kernel_ms(b, ms, &runs) == RSAPRNG_OK && runs == 3, "kernel_ms");
        o.verify(v, "timed eager runs");
        CHECK(rsaprng_batch_check(b) == RSAPRNG_OK, "batch_check");
        rsaprng_batch_destroy(b);
        checked += (long)total * 3;
      }
    CHECK(fakehip::live_device_allocations() == d0 && fakehip::live_streams() == s0 &&
              fakehip::live_events() == e0,
          "batches left device objects behind");
  }

  // 5. the autotuner, generate and consume, through its cache
  {
    uint64_t total;
    auto v = uneven(120, 300, 4, 12, &total);
    auto pr = pool_reqs(v);
    Outputs o(total);
    const size_t d0 = fakehip::live_device_allocations(), s0 = fakehip::live_streams(),
                 e0 = fakehip::live_events();
    rsaprng_config best;
    double ms = 0;
    CHECK(rsaprng_autotune(pool, pr.data(), pr.size(), 0, o.c, o.r, nullptr, cache, st, &best,
                           &ms) == RSAPRNG_OK,
          "autotune generate");
    o.verify(v, "after autotune", 0xA5A5A5A5A5A5A5A5ull);  // the autotuner's own fill
    rsaprng_config again;
    CHECK(rsaprng_autotune(pool, pr.data(), pr.size(), 0, o.c, o.r, nullptr, cache, st, &again,
                           &ms) == RSAPRNG_OK &&
              std::memcmp(&best, &again, sizeof(best)) == 0,
          "autotune cache");
    auto pc = pool_reqs(v, true);
    rsaprng_stats* stats;
    CHECK(hipMalloc(&stats, v.size() * sizeof(rsaprng_stats)) == hipSuccess, "stats");
    CHECK(rsaprng_autotune(pool, pc.data(), pc.size(), 1, nullptr, nullptr, stats, nullptr, st,
                           &best, &ms) == RSAPRNG_OK,
          "autotune consume");
    rsaprng_batch_t b;
    CHECK(rsaprng_batch_create(pool, pc.data(), pc.size(), 1, nullptr, nullptr, stats, &best, st,
                               &b) == RSAPRNG_OK,
          "consume batch after autotune");
    for (int i = 0; i < 3; ++i) CHECK(rsaprng_batch_run(b, st) == RSAPRNG_OK, "batch_run");
    rsaprng_batch_destroy(b);
    CHECK(hipFree(stats) == hipSuccess, "free stats");
    CHECK(fakehip::live_device_allocations() == d0 && fakehip::live_streams() == s0 &&
              fakehip::live_events() == e0,
          "autotune left device objects behind");
  }

  // 6. the server: requests arriving in waves, read back and released; then a
  //    replay.  Two passes with 8 indices per lane, then with 16 (iterations
  //    grouped by exponent class)
  for (int per : {8, 16}) {
    const size_t d0 = fakehip::live_device_allocations(), s0 = fakehip::live_streams(),
                 e0 = fakehip::live_events();
    rsaprng_server_opts opts;
    std::memset(&opts, 0, sizeof(opts));
    opts.arena_bytes = (size_t)16 << 20;  // 2^20 outputs
    opts.iter_outputs = 1 << 16;
    opts.chunk_outputs = 1 << 14;
    opts.cfg = cfg_of(2, 0, 256, 2, 0, per);
    rsaprng_server_t srv;
    CHECK(rsaprng_server_create(pool, &opts, &srv) == RSAPRNG_OK, "server_create");
    uint64_t total;
    auto v = uneven(200, 300, 6, 17, &total);
    size_t done = 0, next = 0;
    std::vector<rsaprng_completion> comp(64);
    std::vector<uint64_t> hc, hr;
    while (done < v.size()) {
      for (int w = 0; w < 25 && next < v.size(); ++w, ++next) {
        const int rc = rsaprng_server_submit(srv, v[next].inst, v[next].k0, v[next].count, next);
        CHECK(rc == RSAPRNG_OK, "server_submit %d", rc);
      }
      const int n = rsaprng_server_poll(srv, comp.data(), comp.size());
      CHECK(n >= 0, "server_poll %d", n);
      for (int i = 0; i < n; ++i) {
        const HReq& q = v[comp[i].tag];
        CHECK(comp[i].count == q.count, "completion count");
        hc.assign(q.count, 0);
        hr.assign(q.count, 0);
        CHECK(rsaprng_server_read(srv, comp[i].tag, 0, q.count, hc.data(),
                                  reinterpret_cast<double*>(hr.data()), nullptr) == RSAPRNG_OK,
              "server_read");
        for (uint64_t j = 0; j < q.count; ++j)
          CHECK(hc[j] == tag_c(q.inst, q.k0 + j) && hr[j] == tag_r(q.inst, q.k0 + j),
                "served request %" PRIu64 " output %" PRIu64 " wrong", comp[i].tag, j);
        CHECK(rsaprng_server_release(srv, comp[i].tag) == RSAPRNG_OK, "server_release");
        ++done;
        checked += (long)q.count;
      }
    }
    std::vector<uint32_t> inst(150);
    std::vector<uint64_t> k0(150), cnt(150);
    std::vector<double> ta(150), tad(150), tdn(150);
    for (size_t i = 0; i < inst.size(); ++i) {
      inst[i] = (uint32_t)(rng() % 300);
      k0[i] = rng() >> 24;
      cnt[i] = 1 + rng() % 50000;
      ta[i] = 1e-4 * (double)i;
    }
    CHECK(rsaprng_server_replay(srv, inst.size(), inst.data(), k0.data(), cnt.data(), ta.data(),
                                tad.data(), tdn.data()) == RSAPRNG_OK,
          "server_replay");
    uint64_t it = 0, outs = 0, wait = 0, act = 0;
    CHECK(rsaprng_server_stats(srv, &it, &outs, &wait, &act) == RSAPRNG_OK && wait == 0 &&
              act == 0,
          "server_stats");
    rsaprng_server_destroy(srv);
    CHECK(fakehip::live_device_allocations() == d0 && fakehip::live_streams() == s0 &&
              fakehip::live_events() == e0,
          "server left device objects behind");
  }

  // 7. single handles, handle batches, vector mode, checks and parameter generation
  {
    rsaprng_t h = rsaprng_create(4294967291ull, 2147483659ull, 7, 12345);
    CHECK(h, "create (%d)", rsaprng_last_error());
    Outputs o(200000);
    for (uint64_t k0 : {0ull, (1ull << 20) - 777, (1ull << 63) + 5, ~0ull - 99999})
      CHECK(rsaprng_generate(h, k0, 100000, o.c, o.r, st) == RSAPRNG_OK, "generate");
    rsaprng_stats* stats;
    CHECK(hipMalloc(&stats, sizeof(rsaprng_stats)) == hipSuccess, "stats");
    CHECK(rsaprng_consume(h, 99, 3 << 20, stats, st) == RSAPRNG_OK, "consume");
    rsaprng_req rq[2] = {{h, 10, 1000, 0}, {h, 5 << 20, 5000, 1000}};
    CHECK(rsaprng_generate_batch(rq, 2, o.c, o.r, st) == RSAPRNG_OK, "generate_batch");
    for (uint64_t mv : {1ull, 8ull, 64ull, 4096ull})
      CHECK(rsaprng_generate_vector(h, mv, 3 * mv + 1, 150000, o.c, o.r, 2, st) == RSAPRNG_OK,
            "generate_vector");
    uint64_t* m;
    CHECK(hipMalloc(&m, 64 * 8) == hipSuccess, "m");
    CHECK(rsaprng_debug_encrypt(1000003, 1000033, 5, 2, m, o.c, o.r, 64, st) == RSAPRNG_OK,
          "debug_encrypt");
    uint64_t count = 0;
    CHECK(rsaprng_prime_count(1ull << 31, (1ull << 31) + 1000, 0, &count, st) == RSAPRNG_OK,
          "prime_count");
    const uint32_t ex[2] = {3, 5};
    CHECK(rsaprng_next_primes(m, 64, 0, ex, 2, o.c, st) == RSAPRNG_OK, "next_primes");
    double work = 0;
    CHECK(rsaprng_probe(RSAPRNG_PROBE_FMA_F64, 4, nullptr, nullptr, &work, st) == RSAPRNG_OK,
          "probe");
    rsaprng_battery* bat;
    CHECK(hipMalloc(&bat, sizeof(rsaprng_battery)) == hipSuccess, "battery");
    uint64_t tb;
    auto vb = uneven(30, 300, 6, 15, &tb);
    auto pb = pool_reqs(vb);
    CHECK(rsaprng_pool_battery(pool, pb.data(), pb.size(), bat, nullptr, st) == RSAPRNG_OK,
          "pool_battery");
    // 16 indices per lane asked of the battery: it runs on lanes of 8
    const rsaprng_config c16 = cfg_of(2, 2, 256, 1, 1, 16);
    CHECK(rsaprng_pool_battery(pool, pb.data(), pb.size(), bat, &c16, st) == RSAPRNG_OK,
          "pool_battery, 16 per lane asked");
    CHECK(rsaprng_battery_values(o.r, 100000, bat, st) == RSAPRNG_OK, "battery_values");
    CHECK(rsaprng_check_device_error(st) == RSAPRNG_OK, "device error");
    fakehip::drain();
    CHECK(hipFree(bat) == hipSuccess && hipFree(m) == hipSuccess && hipFree(stats) == hipSuccess,
          "free");
    rsaprng_destroy(h);
  }

  rsaprng_pool_destroy(pool);
  rsaprng_pool_destroy(pool3);
  CHECK(hipStreamDestroy(st) == hipSuccess, "stream");
  std::printf("ok %ld outputs checked\n", checked);
  return 0;
}
