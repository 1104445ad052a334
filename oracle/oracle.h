/*
 * Plain CPU oracle for the RSA-exponentiation pseudorandom generator of
 * Datephanyawat & Beale, "A class of scalable parallel and vectorizable
 * pseudorandom number generators based on non-cryptographic RSA exponentiation
 * ciphers" (arXiv:1811.11629).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this code; only the tests, the smoke check and the benchmark's CPU
 * baseline leg do.  It shares no source, header, table or helper with the GPU
 * path.  Arithmetic is deliberately the slowest obviously-correct form:
 * 128-bit products reduced with '%', binary exponentiation, and C's own
 * integer->double conversion and IEEE division.
 *
 * Definition computed (sequence of instance (p, q, e, m0, s0)):
 *   Q = 2^63 - 25, a = 2307085864                      (Implementation section)
 *   s_j = s0 * a^j mod Q                                 (eq. congruentialgenerator1)
 *   within block b = floor(k / B), B = 2^20:
 *     m_k = (m0 + G_b + sum_{j=bB+1..k} s_j) mod n,      (skip recurrence m_k = m_{k-1}+s_k)
 *     G_b = (sum_{j=1..bB} s_j) mod Q   (closed form of a geometric series, eq. pseudoskip)
 *   c_k = m_k^e mod n                                    (eq. encrypt2)
 *   r_k = RN(RN(c_k) / RN(n)); r_k = 1 - 2^-53 if that equals 1.0   (r = c/n, and the
 *         guard against returning 1.0 required after algorithm (1))
 * For k < 2^20 this is exactly the paper's recurrence started from (m0, s0).
 * Block re-seeding at multiples of 2^20 is this project's reading of how to jump
 * the message sequence, which the paper leaves open (the closed form in
 * eq. pseudoskip is laborious to evaluate except near multiples of Q-1).
 */
#ifndef RSAPRNG_ORACLE_H
#define RSAPRNG_ORACLE_H
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif

#define ORACLE_Q 9223372036854775783ULL /* 2^63 - 25 */
#define ORACLE_A 2307085864ULL          /* primitive root recommended by L'Ecuyer et al. */
#define ORACLE_BLOCK_LOG2 20

uint64_t oracle_mulmod(uint64_t x, uint64_t y, uint64_t m);
uint64_t oracle_powmod(uint64_t x, uint64_t e, uint64_t m);
uint64_t oracle_gcd(uint64_t x, uint64_t y);
/* x^-1 mod m by the extended Euclidean algorithm; 0 if none exists. */
uint64_t oracle_inverse(uint64_t x, uint64_t m);
/* Miller-Rabin after trial division: the 12 smallest prime bases below 2^64,
 * the 5 smallest below 2^32 (Implementation section). */
int oracle_is_prime(uint64_t n);
/* Parameter rule: 0 if (p, q, e) is usable, else a negative code
 * (-1 not prime, -2 p == q, -3 outside [2^31, 2^32), -4 bad exponent). */
int oracle_check_params(uint64_t p, uint64_t q, uint64_t e);
/* Decryption exponent d = e^-1 mod phi(n) (use_lambda = 0) or mod lambda(n). */
uint64_t oracle_decryption_exponent(uint64_t p, uint64_t q, uint64_t e, int use_lambda);

/* One skip step a*s mod Q: with a 128-bit product, and with the paper's
 * restricted-primitive-root (Schrage) decomposition Q = a*q1 + q2. */
uint64_t oracle_lcg_next(uint64_t s);
uint64_t oracle_lcg_next_schrage(uint64_t s);
/* s0 * a^k mod Q */
uint64_t oracle_skip(uint64_t s0, uint64_t k);
/* G_b by the closed form s0*a*(a^{bB}-1)/(a-1) mod Q */
uint64_t oracle_block_seed(uint64_t s0, uint64_t b);
/* G_b by walking: (sum of s_1..s_{bB} as an exact integer) mod Q.  O(bB). */
uint64_t oracle_block_seed_walk(uint64_t s0, uint64_t b);

/* r = RN(c)/RN(n) with the 1.0 guard. */
double oracle_ratio(uint64_t c, uint64_t n);

/* Outputs c_k (and r_k) for k in [k0, k0+count) of instance (p, q, e, m0, s0).
 * Either output pointer may be NULL.  Returns 0, or a negative code for bad
 * parameters (m0 must be < n, 1 <= s0 < Q). */
int oracle_generate(uint64_t p, uint64_t q, uint64_t e, uint64_t m0, uint64_t s0,
                    uint64_t k0, uint64_t count, uint64_t* c_out, double* r_out);

/* Messages m_k (before encryption) for k in [k0, k0+count). */
int oracle_messages(uint64_t p, uint64_t q, uint64_t m0, uint64_t s0,
                    uint64_t k0, uint64_t count, uint64_t* m_out);

/* Algorithm (1) as the paper states it: Schrage skip step, CRT residues,
 * two exponentiations mod the 32-bit primes, Garner recombination and the
 * division.  Returns the first `count` numbers a caller receives, i.e.
 * c_1, c_2, ... (the state starts at (m0, s0)); no block re-seeding. */
int oracle_paper_algorithm1(uint64_t p, uint64_t q, uint64_t e, uint64_t m0, uint64_t s0,
                            uint64_t count, uint64_t* c_out, double* r_out);

/* c = m^e mod n for each element (any odd n >= 3). */
void oracle_encrypt_array(uint64_t n, uint64_t e, const uint64_t* m, uint64_t* c, uint64_t count);

/* Statistics of r_k over k in [k0, k0+count):
 *   sum_fx[0..2]: exact sum of r_k as a 192-bit fixed-point number with its
 *                 least significant bit worth 2^-128 (little-endian limbs);
 *   lt_half:      number of r_k < 0.5;
 *   hist[1024]:   hist[floor(1024 r_k)] counts.                                  */
typedef struct {
  uint64_t sum_fx[3];
  uint64_t lt_half;
  uint64_t hist[1024];
} oracle_stats;
int oracle_consume(uint64_t p, uint64_t q, uint64_t e, uint64_t m0, uint64_t s0,
                   uint64_t k0, uint64_t count, oracle_stats* st);
/* Same statistics over a given array of r values. */
void oracle_stats_of(const double* r, uint64_t count, oracle_stats* st);

/* Parameter generation (Implementation section).  Number of primes, or safe
 * primes p = 2 p' + 1 with p' prime, in [lo, hi) for hi <= 2^32, by a segmented
 * sieve; and the smallest p >= x below 2^32 that is prime (safe if asked) with
 * p mod f != 1 for every listed f, or 0. */
uint64_t oracle_count_primes(uint64_t lo, uint64_t hi, int safe);
uint64_t oracle_next_prime(uint64_t x, int safe, const uint32_t* exps, int nexp);

/* Statistical battery (Tests section: frequency with 2^20 bins, serial tests
 * in D = 2..6 dimensions, poker with five cards of sixteen denominations,
 * maximum of t = 32).  Groups: inside aligned blocks of 8 absolute indices
 * (8j .. 8j+7) the D-tuples at offsets 0, D, 2D, ... that fit, and the poker
 * hand at offsets 0..4; aligned blocks of 32 for the maximum; only blocks whose
 * indices all lie in [k0, k0+count) count.  Bin of r with b bins per
 * coordinate: min(floor(b r), b - 1); a serial cell is the mixed-radix number
 * of its coordinates, first index most significant; the poker class is the
 * number of distinct floor(16 r); the maximum M goes to floor(1024 M^32) with
 * M^32 by five squarings.  Collision test: each aligned block of 2^14
 * indices throws 2^14 balls into 2^20 urns floor(2^20 r); C = 2^14 minus the
 * number of distinct urns, counted in coll[min(C, 255)].  Gaps test (runs of
 * 0s and 1s with b = [r > 1/2]): in each aligned block of 64 indices the run
 * starting at its first index, value b and length L <= 64, in runs[b][L - 1].
 * Collision test on leading bits: inside each block of 2^20 indices, balls of
 * 20 consecutive indices from the block's start (20 g .. 20 g + 19 relative
 * to it), the urn the 20-bit number whose bit j is the leading bit
 * floor(2 r) of the ball's j-th value; trials of 2^14 consecutive balls, the
 * first three of the block (its last 65536 indices take no ball); a trial
 * whose indices all lie in [k0, k0+count) counts 2^14 minus its distinct urns
 * in coll_msb[min(C, 255)].
 * oracle_battery_add ACCUMULATES into *b. */
typedef struct {
  uint64_t outputs;
  uint64_t reserved;
  uint32_t freq[1 << 20];
  uint32_t serial2[1 << 20];
  uint32_t serial3[1000000];
  uint32_t serial4[1 << 20];
  uint32_t serial5[1 << 20];
  uint32_t serial6[1000000];
  uint32_t poker[8];
  uint32_t maxt[1024];
  uint32_t coll[256];
  uint32_t runs[2][64];
  uint32_t coll_msb[256];
} oracle_battery;
int oracle_battery_add(uint64_t p, uint64_t q, uint64_t e, uint64_t m0, uint64_t s0, uint64_t k0,
                       uint64_t count, oracle_battery* b);
/* The same counts over given values r[0 .. count) standing at absolute indices
 * k0 .. k0 + count - 1 (the groups are aligned to those indices); ACCUMULATES. */
int oracle_battery_values(const double* r, uint64_t k0, uint64_t count, oracle_battery* b);

#ifdef __cplusplus
}
#endif
#endif
