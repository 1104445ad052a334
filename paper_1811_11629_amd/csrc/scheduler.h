// Scheduling core of the served form: admission by output-arena space and
// continuation slots, and iteration-level chunking of admitted requests.  It
// touches no device: the server drives it from its request loop, and a
// host-only dry run drives it for tests.
#pragma once
#include <algorithm>
#include <cstring>
#include <deque>
#include <map>
#include <vector>

#include "common.h"
#include "plan.h"

namespace rsaprng {

// First-fit allocator over [0, size) in output elements; adjacent free ranges
// are merged on release.
class Arena {
 public:
  explicit Arena(u64h size) : size_(size) {
    if (size) free_[0] = size;
  }
  bool alloc(u64h len, u64h* off) {
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= len) {
        *off = it->first;
        const u64h rest = it->second - len, start = it->first + len;
        free_.erase(it);
        if (rest) free_[start] = rest;
        used_ += len;
        return true;
      }
    }
    return false;
  }
  void release(u64h off, u64h len) {
    used_ -= len;
    auto it = free_.emplace(off, len).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
  u64h size() const { return size_; }
  u64h used() const { return used_; }

 private:
  u64h size_, used_ = 0;
  std::map<u64h, u64h> free_;
};

enum SrvState { kSrvWaiting = 0, kSrvActive = 1, kSrvDone = 2 };
// Order in which an iteration takes the admitted requests' next chunks.
enum SrvPolicy { kSrvRoundRobin = 0, kSrvShortestFirst = 1 };

struct SrvReq {
  uint64_t tag = 0;
  uint32_t inst = 0, e = 0;
  u64h k0 = 0, count = 0;
  u64h pos = 0;          // next index to schedule
  u64h off = 0;          // arena offset of output k0
  uint32_t slot = 0;     // continuation state slot
  int state = kSrvWaiting;
  bool scheduled_all = false;
  double t_submit = 0, t_admit = 0, t_done = 0;
};

class Scheduler {
 public:
  // T: tile size of the kernel configuration (a power of two dividing 2^20).
  // Every chunk but a request's last ends on a multiple of T, so the next chunk
  // can start from the chain state at a tile boundary.
  Scheduler(u64h arena_elems, uint32_t nslots, u64h T, u64h iter_outputs, u64h chunk_outputs,
            int policy = kSrvRoundRobin)
      : arena_(arena_elems), T_(T), policy_(policy) {
    chunk_ = std::max<u64h>(chunk_outputs, T);
    iter_ = std::max<u64h>(iter_outputs, chunk_);
    free_slots_.resize(nslots);
    for (uint32_t i = 0; i < nslots; ++i) free_slots_[i] = nslots - 1 - i;
  }

  void enqueue(SrvReq* r) { waiting_.push_back(r); }

  // FIFO admission while the head request's outputs fit in the arena and a
  // slot is free (the head blocks later arrivals, so none starves).
  void admit(double t) {
    while (!waiting_.empty() && !free_slots_.empty()) {
      SrvReq* r = waiting_.front();
      u64h off;
      if (!arena_.alloc(r->count, &off)) break;
      r->off = off;
      r->slot = free_slots_.back();
      free_slots_.pop_back();
      r->state = kSrvActive;
      r->t_admit = t;
      active_.push_back(r);
      waiting_.pop_front();
    }
  }

  // The next iteration: at most one chunk per admitted request, up to iter
  // outputs in all.  Round robin: an iteration starts after the last request
  // the previous one planned.  Shortest first: the requests with the fewest
  // outputs left go first (admission order between equals), which keeps most
  // requests, the short ones, from waiting behind long ones.  Returns false if
  // there is nothing to run.  Requests whose last chunk is planned go to
  // `finishing`.
  bool plan(std::vector<PlanIn>& out, std::vector<SrvReq*>& finishing, u64h* total) {
    out.clear();
    finishing.clear();
    u64h budget = iter_, sum = 0;
    const size_t na = active_.size();
    size_t next_rr = rr_;
    const bool sf = policy_ == kSrvShortestFirst;
    if (sf) {
      order_.clear();
      for (size_t i = 0; i < na; ++i)
        if (!active_[i]->scheduled_all) order_.push_back(active_[i]);
      std::stable_sort(order_.begin(), order_.end(), [](const SrvReq* a, const SrvReq* b) {
        return left(a) < left(b);
      });
    }
    const size_t n_try = sf ? order_.size() : na;
    for (size_t i = 0; i < n_try && budget > 0; ++i) {
      SrvReq* r = sf ? order_[i] : active_[(rr_ + i) % na];
      if (r->scheduled_all) continue;
      const u64h remaining = left(r);
      u64h len = std::min(std::min(remaining, chunk_), budget);
      if (len < remaining) {
        const u64h end = (r->pos + len) & ~(T_ - 1);
        if (end > r->pos) {
          len = end - r->pos;
        } else {
          // shorter than the distance to the next tile boundary
          len = std::min(T_ - (r->pos & (T_ - 1)), remaining);
          if (len > budget) continue;
        }
      }
      PlanIn in;
      std::memset(&in, 0, sizeof(in));
      in.inst = r->inst;
      in.e = r->e;
      in.k0 = r->pos;
      in.count = len;
      in.out_off = r->off + (r->pos - r->k0);
      in.slot = r->slot;
      const bool last = len == remaining;
      const u64h next = r->pos + len;
      if (r->pos != r->k0 && (r->pos & (kBlock - 1)) != 0) {
        in.flags |= kReqContinue;
        in.S = r->pos;
      }
      if (!last && (next & (kBlock - 1)) != 0) in.flags |= kReqWriteEnd;
      out.push_back(in);
      if (!sf) next_rr = rr_ + i + 1;
      r->pos = next;
      budget -= len;
      sum += len;
      if (last) {
        r->scheduled_all = true;
        finishing.push_back(r);
      }
    }
    // the next iteration starts after the last request planned here
    rr_ = na ? next_rr % na : 0;
    *total = sum;
    return !out.empty();
  }

  void finish(SrvReq* r, double t) {
    r->state = kSrvDone;
    r->t_done = t;
    active_.erase(std::find(active_.begin(), active_.end(), r));
  }

  void release(SrvReq* r) {
    arena_.release(r->off, r->count);
    free_slots_.push_back(r->slot);
  }

  // outputs of r not yet planned; mod 2^64, since k0 + count may be 2^64
  static u64h left(const SrvReq* r) { return (r->k0 + r->count) - r->pos; }

  size_t waiting() const { return waiting_.size(); }
  size_t active() const { return active_.size(); }
  u64h arena_size() const { return arena_.size(); }

 private:
  Arena arena_;
  u64h T_, chunk_, iter_;
  int policy_;
  std::vector<SrvReq*> order_;  // shortest first: this iteration's order
  std::vector<uint32_t> free_slots_;
  std::deque<SrvReq*> waiting_;
  std::vector<SrvReq*> active_;
  size_t rr_ = 0;
};

}  // namespace rsaprng
