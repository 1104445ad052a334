/* Workload-generation helper: for each query x in [2^31, 2^32), the smallest
 * prime P >= x with P mod f != 1 for every listed exponent f, or 0 if there is
 * none up to 2^32.  A segmented sieve of Eratosthenes over the odd numbers of
 * [2^31, 2^32) with every prime below 2^16 -- the same definition of primality
 * as trial division, at a fraction of the cost for large workloads.  Holds no
 * arithmetic of the generator. */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define LO 2147483649ULL          /* 2^31 + 1, first odd number of the range */
#define NODD (1ULL << 30)         /* odd numbers in [2^31, 2^32) */
#define SEG (1u << 18)            /* odd numbers per segment */

static int cmp_u64(const void* a, const void* b) {
  uint64_t x = *(const uint64_t*)a, y = *(const uint64_t*)b;
  return x < y ? -1 : x > y;
}

/* queries[i] < 2^32; answers written in the order of the queries.  Returns 0 or -1. */
int next_primes(const uint64_t* queries, uint64_t n, const uint32_t* exps, int nexps,
                uint64_t* answers) {
  /* small primes below 2^16 */
  static uint32_t small[6542];
  int ns = 0;
  {
    static unsigned char comp[1 << 16];
    memset(comp, 0, sizeof(comp));
    for (uint32_t i = 2; i < (1u << 16); ++i) {
      if (comp[i]) continue;
      small[ns++] = i;
      for (uint32_t j = i * i; j < (1u << 16); j += i) comp[j] = 1;
    }
  }
  /* queries sorted by value, remembering their positions */
  uint64_t* key = (uint64_t*)malloc(n * 16 + 16);
  unsigned char* seg = (unsigned char*)malloc(SEG);
  if (!key || !seg) {
    free(key);
    free(seg);
    return -1;
  }
  for (uint64_t i = 0; i < n; ++i) {
    key[2 * i] = queries[i];
    key[2 * i + 1] = i;
    answers[i] = 0;
  }
  qsort(key, n, 16, cmp_u64);
  uint64_t qi = 0;
  while (qi < n && key[2 * qi] <= 2) ++qi; /* not in range: answer 0 */
  for (uint64_t s0 = 0; s0 < NODD && qi < n; s0 += SEG) {
    const uint64_t lo = LO + 2 * s0; /* number at index s0 */
    const uint64_t hi = lo + 2 * (uint64_t)(SEG - 1);
    if (hi < key[2 * qi]) continue; /* no pending query reaches this segment */
    memset(seg, 1, SEG);
    for (int k = 1; k < ns; ++k) { /* odd primes */
      const uint64_t p = small[k];
      uint64_t m = (lo + p - 1) / p * p;
      if ((m & 1) == 0) m += p;
      for (uint64_t j = (m - lo) / 2; j < SEG; j += p) seg[j] = 0;
    }
    for (uint32_t j = 0; j < SEG && qi < n; ++j) {
      if (!seg[j]) continue;
      const uint64_t P = lo + 2 * (uint64_t)j;
      int ok = 1;
      for (int f = 0; f < nexps; ++f)
        if (P % exps[f] == 1) ok = 0;
      if (!ok) continue;
      while (qi < n && key[2 * qi] <= P) {
        answers[key[2 * qi + 1]] = P;
        ++qi;
      }
    }
  }
  free(key);
  free(seg);
  return 0;
}
