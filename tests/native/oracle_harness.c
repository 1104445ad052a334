/* Driver of the CPU oracle (oracle/oracle.c) for sanitizer builds: generation,
 * consumption, the battery and prime counts on small ranges, printed as
 * 64-bit digests of the results. */
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

static uint64_t fnv(uint64_t h, const void* p, size_t n) {
  const unsigned char* b = (const unsigned char*)p;
  for (size_t i = 0; i < n; ++i) {
    h ^= b[i];
    h *= 1099511628211ull;
  }
  return h;
}

int main(void) {
  const uint64_t p = 2147483693ull, q = 2147483777ull, e = 3, m0 = 12345;
  const uint64_t cnt = 40000;
  uint64_t* c = malloc(cnt * sizeof(uint64_t));
  double* r = malloc(cnt * sizeof(double));
  oracle_battery* B = calloc(1, sizeof(oracle_battery));
  if (!c || !r || !B) return 2;
  const uint64_t k0s[3] = {0, (1ull << 20) - 1000, (1ull << 63) + 7};
  uint64_t h = 14695981039346656037ull;
  for (int i = 0; i < 3; ++i) {
    if (oracle_generate(p, q, e, m0, 1, k0s[i], cnt, c, r)) return 3;
    h = fnv(h, c, cnt * sizeof(uint64_t));
    h = fnv(h, r, cnt * sizeof(double));
    if (oracle_battery_add(p, q, e, m0, 1, k0s[i], cnt, B)) return 4;
  }
  printf("generate %016llx\n", (unsigned long long)h);
  /* the record as 32-bit words, sum of (i + 1) w_i mod 2^64 */
  const uint32_t* w = (const uint32_t*)B;
  uint64_t bs = 0;
  for (size_t i = 0; i < sizeof(*B) / 4; ++i) bs += (uint64_t)(i + 1) * w[i];
  printf("battery %016llx\n", (unsigned long long)bs);
  printf("primes %llu %llu\n", (unsigned long long)oracle_count_primes(2147483648ull, 2147483648ull + 200000, 0),
         (unsigned long long)oracle_count_primes(2147483648ull, 2147483648ull + 200000, 1));
  free(c);
  free(r);
  free(B);
  return 0;
}
