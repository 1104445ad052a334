// Host build of the library's 32-bit primality code (the same header the
// prime kernels include), for checking it exhaustively against the oracle.
#define RSAPRNG_HD inline
#include "primes.h"

using namespace rsaprng;

extern "C" uint64_t harness_count(uint64_t lo, uint64_t hi, int safe) {
  const SmallPrimeTable sp = make_small_primes();
  if (lo >= hi) return 0;
  uint64_t c = count_small(lo, hi, safe != 0);
  for (uint64_t row = lo / 30; row < (hi + 29) / 30; ++row) c += count_row(row, lo, hi, safe != 0, sp);
  return c;
}

extern "C" int harness_is_prime(uint32_t n) {
  const SmallPrimeTable sp = make_small_primes();
  return is_prime32(n, sp.p) ? 1 : 0;
}
