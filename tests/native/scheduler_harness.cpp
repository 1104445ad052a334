// Host-only driver of the served form's scheduler (paper_1811_11629_amd/csrc/
// scheduler.h) for sanitizer builds: random arenas, slot counts, tile sizes and
// request streams, with the invariants the server relies on checked after
// every iteration.  Prints "ok <iterations>" or the first violation.
#include <cstdio>
#include <cstdlib>
#include <memory>
#include <random>
#include <vector>

#include "scheduler.h"

using namespace rsaprng;

#define CHECK(c, ...)                      \
  do {                                     \
    if (!(c)) {                            \
      std::printf("violation: " __VA_ARGS__); \
      std::printf("\n");                   \
      return 1;                            \
    }                                      \
  } while (0)

int main(int argc, char** argv) {
  const unsigned seed = argc > 1 ? (unsigned)std::atoi(argv[1]) : 1u;
  std::mt19937_64 rng(seed);
  long iterations = 0;
  for (int trial = 0; trial < 40; ++trial) {
    const u64h arena = 1ull << (12 + rng() % 10);
    const uint32_t nslots = 1 + rng() % 48;
    const u64h T = 1ull << (8 + rng() % 6);
    const u64h iter = T * (1 + rng() % 64), chunk = T * (1 + rng() % 16);
    // both policies, alternately
    Scheduler sc(arena, nslots, T, iter, chunk, trial % 2 ? kSrvShortestFirst : kSrvRoundRobin);
    const u64h budget = std::max(iter, std::max(chunk, T));  // the scheduler's own rounding
    const int nreq = 150;
    std::vector<std::unique_ptr<SrvReq>> reqs;
    std::vector<u64h> next(nreq), arrive(nreq);
    for (int i = 0; i < nreq; ++i) {
      auto r = std::make_unique<SrvReq>();
      r->tag = i;
      r->inst = (uint32_t)(rng() % 1000);
      r->e = 3;
      r->count = 1 + rng() % arena;
      switch (rng() % 4) {  // starts: block-aligned, ragged, deep, at the top of the index range
        case 0: r->k0 = (rng() % 64) << kBlockLog2; break;
        case 1: r->k0 = rng() % (1ull << 24); break;
        case 2: r->k0 = rng() >> 20; break;
        default: r->k0 = 0ull - r->count; break;  // k0 + count = 2^64
      }
      r->pos = r->k0;
      next[i] = r->k0;
      arrive[i] = rng() % 200;
      reqs.push_back(std::move(r));
    }
    int done = 0;
    std::vector<PlanIn> plan;
    std::vector<SrvReq*> fin;
    for (u64h it = 0; done < nreq; ++it) {
      CHECK(it < 1000000, "no progress (trial %d)", trial);
      for (int i = 0; i < nreq; ++i)
        if (arrive[i] == it) sc.enqueue(reqs[i].get());
      sc.admit((double)it);
      // admitted outputs: disjoint ranges inside the arena, distinct slots
      std::vector<std::pair<u64h, u64h>> rg;
      std::vector<int> slot_used(nslots, 0);
      for (auto& r : reqs)
        if (r->state == kSrvActive) {
          CHECK(r->off + r->count <= arena, "range outside the arena");
          rg.push_back({r->off, r->off + r->count});
          CHECK(r->slot < nslots && !slot_used[r->slot]++, "slot reused");
        }
      std::sort(rg.begin(), rg.end());
      for (size_t j = 1; j < rg.size(); ++j) CHECK(rg[j - 1].second <= rg[j].first, "arena overlap");
      u64h total = 0;
      if (!sc.plan(plan, fin, &total)) continue;
      ++iterations;
      u64h sum = 0;
      CHECK(total <= budget, "iteration over budget");
      for (const PlanIn& in : plan) {
        SrvReq* r = nullptr;
        for (auto& q : reqs)
          if (q->state == kSrvActive && q->slot == in.slot) r = q.get();
        CHECK(r, "chunk of no active request");
        const int i = (int)r->tag;
        CHECK(in.k0 == next[i] && in.count > 0, "chunk out of order");
        CHECK(in.out_off == r->off + (in.k0 - r->k0), "wrong output offset");
        const u64h end = in.k0 + in.count;  // mod 2^64
        const bool last = end == r->k0 + r->count;
        CHECK(last || (end & (T - 1)) == 0, "chunk end not tile-aligned");
        const bool cont = in.k0 != r->k0 && (in.k0 & (kBlock - 1)) != 0;
        CHECK(!!(in.flags & kReqContinue) == cont, "continuation flag");
        CHECK(!(cont && in.S != in.k0), "continuation start");
        CHECK(!!(in.flags & kReqWriteEnd) == (!last && (end & (kBlock - 1)) != 0), "write-end flag");
        next[i] = end;
        sum += in.count;
      }
      CHECK(sum == total, "total");
      for (SrvReq* r : fin) {
        CHECK(next[r->tag] == r->k0 + r->count, "finished before its last index");
        sc.finish(r, (double)it);
        sc.release(r);
        ++done;
      }
    }
  }
  std::printf("ok %ld\n", iterations);
  return 0;
}
