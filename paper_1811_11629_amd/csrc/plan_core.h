// Planning steps shared by every launch path: when consecutive requests form
// one index range, the tile range of a request, and the chains (a request's
// tiles inside one 2^20 block) it splits into.  Host only; nothing here
// allocates, so the no-allocation entry point plans with the same steps.
#pragma once
#include <string.h>

#include "common.h"
#include "plan.h"

namespace rsaprng {

// Requests of one instance that continue each other -- next k0 = previous
// end, and (generate) next output offset = previous end, or (other modes) the
// same statistics record -- are one contiguous range: they share one scan
// chain.  m is the range built so far, r the next request.
inline bool plan_merges(const PlanIn& m, const PlanIn& r, int mode) {
  const bool plain = !(m.flags | r.flags);
  const bool adj_k = m.count && r.k0 == m.k0 + m.count && r.k0 > m.k0;
  const bool adj_o = mode != kModeGenerate ? r.slot == m.slot : r.out_off == m.out_off + m.count;
  // the battery takes requests one by one (a group that only the union of two
  // requests covers is not counted), so it merges none
  return mode != kModeBattery && plain && r.inst == m.inst && adj_k && adj_o && r.count;
}

// The launch record of request r (count > 0) whose tiles, T indices each from
// its scan start S, are numbered from tiles_before.  *nt receives their number.
inline int plan_one(const PlanIn& r, u64h T, u64h tiles_before, Req& q, u64h* nt) {
  if (r.count - 1 > ~0ull - r.k0) return RSAPRNG_E_RANGE;
  memset(&q, 0, sizeof(q));
  q.k0 = r.k0;
  q.count = r.count;
  q.out_off = r.out_off;
  q.inst = r.inst;
  q.slot = r.slot;
  q.flags = r.flags;
  if (r.flags & kReqContinue) {
    if (r.S % T || r.S > r.k0) return RSAPRNG_E_ARG;
    q.S = r.S;
  } else {
    q.S = r.k0 & ~(kBlock - 1);
  }
  const u64h last = r.k0 + (r.count - 1);
  *nt = (last - q.S) / T + 1;
  if (tiles_before + *nt > 0xffffffffull) return RSAPRNG_E_RANGE;
  q.tile_begin = (uint32_t)tiles_before;
  return RSAPRNG_OK;
}

// Calls emit(const Chain&) for every chain of r in index order: one per 2^20
// block that r's tiles touch, each holding r's tiles inside that block.
template <class Emit>
inline void plan_emit_chains(const Req& r, u64h T, Emit&& emit) {
  const u64h last = r.k0 + (r.count - 1);
  u64h x = r.S;
  u64h first = r.tile_begin;
  for (;;) {
    const u64h be = (x & ~(kBlock - 1)) + (kBlock - 1);
    const u64h chain_last = last < be ? last : be;
    const u64h nt = (chain_last - x) / T + 1;
    Chain ch;
    memset(&ch, 0, sizeof(ch));
    ch.S = x;
    ch.k0 = r.k0;
    ch.last = last;
    ch.out_off = r.out_off;
    ch.inst = r.inst;
    ch.first = (uint32_t)first;
    ch.ntiles = (uint32_t)nt;
    ch.slot = r.slot;
    ch.flags = ((r.flags & kReqContinue) && x == r.S ? kChainFromState : 0u) |
               ((r.flags & kReqWriteEnd) && last <= be ? kChainWriteEnd : 0u);
    emit(ch);
    first += nt;
    if (last <= be) break;
    x = be + 1;
  }
}

// Splits the whole tiles before each request's first index off the chains of
// a chain-serial generate launch (the chain-serial kernel would walk them one
// step at a time inside one work-group; the two-pass prefix kernels walk them
// with a wave per tile).  chains[0, n) are the planned chains over `ntiles`
// tiles of T indices; on return chains[0, n) are the output chains (the split
// ones start at their first tile with outputs, flagged kChainStartGiven) and
// chains[n, n + nlead) the lead-in chains, whose slot is the index of their
// output chain.  Lead-in tiles are numbered [0, lead_tiles), the output chains'
// tiles [lead_tiles, ntiles).  Returns RSAPRNG_E_TOO_LARGE if n + nlead
// exceeds cap (nothing is changed then).
inline int plan_split_leadin(Chain* chains, size_t n, size_t cap, u64h T, LeadIn* li) {
  size_t nlead = 0;
  for (size_t i = 0; i < n; ++i) {
    const Chain& C = chains[i];
    if (!(C.flags & kChainFromState) && C.k0 > C.S && (C.k0 - C.S) / T > 0) ++nlead;
  }
  li->nout = (uint32_t)n;
  li->nlead = 0;
  li->lead_tiles = 0;
  if (nlead == 0) return RSAPRNG_OK;
  if (n + nlead > cap || n + nlead > 0xffffffffull) return RSAPRNG_E_TOO_LARGE;
  u64h lead_first = 0;
  for (size_t i = 0; i < n; ++i) {
    const Chain& C = chains[i];
    if (!(C.flags & kChainFromState) && C.k0 > C.S && (C.k0 - C.S) / T > 0)
      lead_first += (C.k0 - C.S) / T;
  }
  const u64h lead_tiles = lead_first;
  u64h lt = 0, ot = lead_tiles;
  size_t l = n;
  for (size_t i = 0; i < n; ++i) {
    Chain& C = chains[i];
    const u64h L = (!(C.flags & kChainFromState) && C.k0 > C.S) ? (C.k0 - C.S) / T : 0;
    if (L > 0) {
      Chain& D = chains[l++];
      memset(&D, 0, sizeof(D));
      D.S = C.S;
      D.k0 = C.S;
      D.last = C.S + L * T - 1;
      D.inst = C.inst;
      D.first = (uint32_t)lt;
      D.ntiles = (uint32_t)L;
      D.slot = (uint32_t)i;
      lt += L;
      C.S += L * T;
      C.ntiles -= (uint32_t)L;
      C.flags |= kChainStartGiven;
    }
    C.first = (uint32_t)ot;
    ot += C.ntiles;
  }
  li->nlead = (uint32_t)nlead;
  li->lead_tiles = lead_tiles;
  return RSAPRNG_OK;
}

}  // namespace rsaprng
