// Primality of 32-bit integers for parameter generation (Implementation
// section: both primes of an instance lie in [2^31, 2^32), the paper
// recommends safe primes p = 2 p' + 1 with p' prime, and the Miller-Rabin
// test with the first five prime bases is deterministic below 2^32).
//
// Arithmetic mod an odd n < 2^32 in Montgomery form with R = 2^32.  The
// functions are __host__ __device__ so that the same code can be checked
// exhaustively on the host.
#pragma once
#include <stdint.h>

namespace rsaprng {

#ifndef RSAPRNG_HD
#define RSAPRNG_HD __host__ __device__ __forceinline__
#endif

struct Mont32 {
  uint32_t n;     // odd modulus
  uint32_t ninv;  // -n^-1 mod 2^32
  uint32_t one;   // R mod n
};

// -n^-1 mod 2^32 by Newton's iteration (each step doubles the correct bits;
// n n = 1 mod 8 gives three to start with).
RSAPRNG_HD uint32_t neg_inv32(uint32_t n) {
  uint32_t x = n;
  x *= 2u - n * x;
  x *= 2u - n * x;
  x *= 2u - n * x;
  x *= 2u - n * x;
  return 0u - x;
}

// a b R^-1 mod n for a, b < n.  t = a b < n^2; with u = t (-n^-1) mod 2^32,
// t + u n is divisible by 2^32 and below 2^65; its low halves sum to 0 mod
// 2^32, carrying exactly when lo32(t) != 0, so the quotient is
// hi(t) + hi(u n) + [lo32(t) != 0] < 2 n, reduced by one subtraction.
RSAPRNG_HD uint32_t mont32_mul(uint32_t a, uint32_t b, const Mont32& M) {
  const uint64_t t = (uint64_t)a * b;
  const uint32_t u = (uint32_t)t * M.ninv;
  const uint64_t un = (uint64_t)u * M.n;
  const uint64_t q = (t >> 32) + (un >> 32) + ((uint32_t)t != 0u);
  return (uint32_t)(q >= M.n ? q - M.n : q);
}

RSAPRNG_HD uint32_t add_mod32(uint32_t a, uint32_t b, uint32_t n) {
  const uint64_t s = (uint64_t)a + b;
  return (uint32_t)(s >= n ? s - n : s);
}

RSAPRNG_HD Mont32 mont32_setup(uint32_t n) {
  Mont32 M;
  M.n = n;
  M.ninv = neg_inv32(n);
  // R mod n: 2^32 - n when n > 2^31, else by division (small moduli only)
  M.one = n > 0x80000000u ? 0u - n : (uint32_t)(0x100000000ull % n);
  return M;
}

// Strong probable-prime test of odd n > 11 to base g < 16, with n - 1 = d 2^s.
RSAPRNG_HD bool sprp32(const Mont32& M, uint32_t g, uint32_t d, int s) {
  // g R mod n by doubling and adding R mod n (g < 16)
  uint32_t gm = 0, pw = M.one;
  for (int b = 0; b < 4; ++b) {
    if ((g >> b) & 1u) gm = add_mod32(gm, pw, M.n);
    pw = add_mod32(pw, pw, M.n);
  }
  // x = g^d in Montgomery form, left to right
  uint32_t x = M.one;
  for (int b = 31; b >= 0; --b) {
    x = mont32_mul(x, x, M);
    if ((d >> b) & 1u) x = mont32_mul(x, gm, M);
  }
  const uint32_t minus_one = M.n - M.one;
  if (x == M.one || x == minus_one) return true;
  for (int i = 1; i < s; ++i) {
    x = mont32_mul(x, x, M);
    if (x == minus_one) return true;
    if (x == M.one) return false;
  }
  return false;
}

// Divisibility of odd n by the odd prime q via q^-1 mod 2^32:
// q | n  <=>  n q^-1 mod 2^32 <= (2^32 - 1) / q.
struct SmallPrime {
  uint32_t q, qinv, lim;
};

RSAPRNG_HD bool divisible(uint32_t n, const SmallPrime& sp) { return n * sp.qinv <= sp.lim; }

// The odd primes below 100 with their inverses mod 2^32 and limits.
constexpr int kSmallPrimes = 24;
struct SmallPrimeTable {
  SmallPrime p[kSmallPrimes];
};
inline SmallPrimeTable make_small_primes() {
  SmallPrimeTable t;
  const uint32_t qs[kSmallPrimes] = {3,  5,  7,  11, 13, 17, 19, 23, 29, 31, 37, 41,
                                     43, 47, 53, 59, 61, 67, 71, 73, 79, 83, 89, 97};
  for (int i = 0; i < kSmallPrimes; ++i) {
    uint32_t x = qs[i];  // q^-1 mod 2^32 by Newton's iteration
    for (int k = 0; k < 5; ++k) x *= 2u - qs[i] * x;
    t.p[i] = SmallPrime{qs[i], x, 0xffffffffu / qs[i]};
  }
  return t;
}

// Deterministic primality for n < 2^32: trial division by the odd primes
// below 100 (with the table), then Miller-Rabin to bases 2, 3, 5, 7, 11.
template <int NSP>
RSAPRNG_HD bool is_prime32(uint32_t n, const SmallPrime (&sp)[NSP]) {
  if (n < 2) return false;
  if ((n & 1u) == 0) return n == 2;
  for (int k = 0; k < NSP; ++k) {
    if (n == sp[k].q) return true;
    if (divisible(n, sp[k])) return false;
  }
  if (n < 97u * 97u) return true;  // no factor below 100 and n < 100^2 (97 is the last prime)
  uint32_t d = n - 1;
  int s = 0;
  while ((d & 1u) == 0) {
    d >>= 1;
    ++s;
  }
  const Mont32 M = mont32_setup(n);
  const uint32_t bases[5] = {2, 3, 5, 7, 11};
  for (int i = 0; i < 5; ++i)
    if (!sprp32(M, bases[i], d, s)) return false;
  return true;
}

// Prime (safe prime when safe) test of a candidate below 2^32.
RSAPRNG_HD bool candidate_ok(uint32_t n, bool safe, const SmallPrimeTable& sp) {
  if (!safe) return is_prime32(n, sp.p);
  // p = 2 p' + 1 with p' prime: beyond 7, p = 3 mod 4 (p' odd) and p = 2 mod 3
  if (n < 8) return n == 5 || n == 7;
  if ((n & 3u) != 3u || n % 3u != 2u) return false;
  return is_prime32((n - 1) >> 1, sp.p) && is_prime32(n, sp.p);
}

// Count over the numbers coprime to 30 in row [30 row, 30 row + 30) that lie
// in [lo, hi).  2, 3 and 5 are not coprime to 30; the caller adds them.
RSAPRNG_HD uint32_t count_row(uint64_t row, uint64_t lo, uint64_t hi, bool safe,
                              const SmallPrimeTable& sp) {
  const uint32_t res[8] = {1, 7, 11, 13, 17, 19, 23, 29};
  uint32_t c = 0;
  const uint64_t base = row * 30;
  for (int k = 0; k < 8; ++k) {
    const uint64_t n = base + res[k];
    if (n >= lo && n < hi && candidate_ok((uint32_t)n, safe, sp)) ++c;
  }
  return c;
}

// The members of {2, 3, 5} in [lo, hi) that count (for safe primes only 5).
RSAPRNG_HD uint32_t count_small(uint64_t lo, uint64_t hi, bool safe) {
  uint32_t c = 0;
  if (!safe) {
    c += (2 >= lo && 2 < hi) + (3 >= lo && 3 < hi);
  }
  c += (5 >= lo && 5 < hi);
  return c;
}

}  // namespace rsaprng
