// A request before planning (host side, no device code): what the planners of
// host.cpp and the served form's scheduler exchange.
#pragma once
#include <stdint.h>

namespace rsaprng {

typedef unsigned long long u64h;

struct PlanIn {
  uint32_t inst;
  uint32_t e;
  u64h k0, count, out_off;
  u64h S;          // continuation scan start (flags & kReqContinue)
  uint32_t slot;
  uint32_t flags;
};

}  // namespace rsaprng
