/*
 * Plain CPU oracle: TEST INFRASTRUCTURE ONLY (see oracle.h for what it computes
 * and which passages of the paper each part follows).  Built with
 * -O2 -ffp-contract=off and no fast-math, so every double operation below is a
 * single IEEE-754 round-to-nearest-even operation.
 */
#include "oracle.h"

#include <math.h>
#include <stddef.h>
#include <stdlib.h>
#include <string.h>

typedef unsigned __int128 u128;

static const uint64_t BLOCK = 1ULL << ORACLE_BLOCK_LOG2;

/* ---- modular arithmetic with 128-bit products (Number Theory section) ---- */

uint64_t oracle_mulmod(uint64_t x, uint64_t y, uint64_t m) {
  return (uint64_t)(((u128)x * y) % m);
}

/* Repeated squaring and multiplying (Introduction: fewer than 2 log2 e products). */
uint64_t oracle_powmod(uint64_t x, uint64_t e, uint64_t m) {
  uint64_t result = 1 % m;
  uint64_t base = x % m;
  while (e) {
    if (e & 1) result = oracle_mulmod(result, base, m);
    base = oracle_mulmod(base, base, m);
    e >>= 1;
  }
  return result;
}

uint64_t oracle_gcd(uint64_t x, uint64_t y) {
  while (y) {
    uint64_t t = x % y;
    x = y;
    y = t;
  }
  return x;
}

/* Extended Euclid on signed 128-bit values (eq. RSAd: d = e^-1 mod phi). */
uint64_t oracle_inverse(uint64_t x, uint64_t m) {
  __int128 r0 = m, r1 = x % m, t0 = 0, t1 = 1;
  while (r1 != 0) {
    __int128 qt = r0 / r1, tmp;
    tmp = r0 - qt * r1; r0 = r1; r1 = tmp;
    tmp = t0 - qt * t1; t0 = t1; t1 = tmp;
  }
  if (r0 != 1) return 0;
  if (t0 < 0) t0 += m;
  return (uint64_t)t0;
}

/* Strong-pseudoprime test to one base g (Implementation section). */
static int strong_probable_prime(uint64_t n, uint64_t g) {
  uint64_t d = n - 1;
  int r = 0;
  while ((d & 1) == 0) { d >>= 1; ++r; }
  uint64_t x = oracle_powmod(g, d, n);
  if (x == 1 || x == n - 1) return 1;
  for (int j = 1; j < r; ++j) {
    x = oracle_mulmod(x, x, n);
    if (x == n - 1) return 1;
  }
  return 0;
}

int oracle_is_prime(uint64_t n) {
  static const uint64_t bases[12] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37};
  if (n < 2) return 0;
  for (int i = 0; i < 12; ++i) {
    if (n == bases[i]) return 1;
    if (n % bases[i] == 0) return 0;
  }
  int nb = (n < (1ULL << 32)) ? 5 : 12;
  for (int i = 0; i < nb; ++i)
    if (!strong_probable_prime(n, bases[i])) return 0;
  return 1;
}

static uint64_t lambda_of(uint64_t p, uint64_t q) {
  uint64_t g = oracle_gcd(p - 1, q - 1);
  return (p - 1) / g * (q - 1);
}

int oracle_check_params(uint64_t p, uint64_t q, uint64_t e) {
  if (p < (1ULL << 31) || p >= (1ULL << 32) || q < (1ULL << 31) || q >= (1ULL << 32)) return -3;
  if (!oracle_is_prime(p) || !oracle_is_prime(q)) return -1;
  if (p == q) return -2;
  /* A decryption exponent exists iff gcd(e, phi) = 1, equivalently gcd(e, lambda) = 1. */
  if (e == 0 || oracle_gcd(e, lambda_of(p, q)) != 1) return -4;
  return 0;
}

uint64_t oracle_decryption_exponent(uint64_t p, uint64_t q, uint64_t e, int use_lambda) {
  uint64_t mod = use_lambda ? lambda_of(p, q) : (p - 1) * (q - 1);
  return oracle_inverse(e, mod);
}

/* ---- skip generator (eq. congruentialgenerator1) ---- */

uint64_t oracle_lcg_next(uint64_t s) { return oracle_mulmod(s, ORACLE_A, ORACLE_Q); }

/* Q = a q1 + q2 with q2 < q1, so both a*(s mod q1) and q2*floor(s/q1) stay
 * below Q (eq. restrictedprimitiveroots); their difference is brought into
 * [0, Q) without going negative. */
uint64_t oracle_lcg_next_schrage(uint64_t s) {
  const uint64_t q1 = ORACLE_Q / ORACLE_A, q2 = ORACLE_Q % ORACLE_A;
  uint64_t s1 = ORACLE_A * (s % q1);
  uint64_t s2 = q2 * (s / q1);
  return (s1 >= s2) ? s1 - s2 : ORACLE_Q - (s2 - s1);
}

uint64_t oracle_skip(uint64_t s0, uint64_t k) {
  return oracle_mulmod(s0, oracle_powmod(ORACLE_A, k, ORACLE_Q), ORACLE_Q);
}

/* sum_{j=1..N} s0 a^j = s0 a (a^N - 1) / (a - 1) in the field Z_Q (eq. pseudoskip). */
uint64_t oracle_block_seed(uint64_t s0, uint64_t b) {
  uint64_t N = b << ORACLE_BLOCK_LOG2;
  uint64_t aN = oracle_powmod(ORACLE_A, N, ORACLE_Q);
  uint64_t num = oracle_mulmod(oracle_mulmod(s0, ORACLE_A, ORACLE_Q), (aN + ORACLE_Q - 1) % ORACLE_Q,
                               ORACLE_Q);
  return oracle_mulmod(num, oracle_inverse(ORACLE_A - 1, ORACLE_Q), ORACLE_Q);
}

uint64_t oracle_block_seed_walk(uint64_t s0, uint64_t b) {
  uint64_t N = b << ORACLE_BLOCK_LOG2;
  uint64_t s = s0;
  u128 sum = 0;
  for (uint64_t j = 1; j <= N; ++j) {
    s = oracle_lcg_next(s);
    sum += s;
  }
  return (uint64_t)(sum % ORACLE_Q);
}

/* ---- floating-point output (eq. CodeFloatingPointStep) ---- */

double oracle_ratio(uint64_t c, uint64_t n) {
  double r = (double)c / (double)n;
  if (r == 1.0) r = nextafter(1.0, 0.0);
  return r;
}

/* ---- the sequence ---- */

static int instance_ok(uint64_t p, uint64_t q, uint64_t e, uint64_t m0, uint64_t s0) {
  int rc = oracle_check_params(p, q, e);
  if (rc) return rc;
  if (m0 >= p * q) return -5;
  if (s0 == 0 || s0 >= ORACLE_Q) return -5;
  return 0;
}

/* Walk the message sequence over [k0, k0+count), calling back with (k, m_k). */
static int walk(uint64_t p, uint64_t q, uint64_t m0, uint64_t s0, uint64_t k0, uint64_t count,
                void (*emit)(void*, uint64_t, uint64_t), void* ctx) {
  if (count == 0) return 0;
  if ((u128)k0 + count > ((u128)1 << 64)) return -6;
  uint64_t n = p * q;
  uint64_t b = k0 >> ORACLE_BLOCK_LOG2;
  uint64_t k = b << ORACLE_BLOCK_LOG2;
  uint64_t s = oracle_skip(s0, k);
  uint64_t m = (uint64_t)(((u128)m0 + oracle_block_seed(s0, b)) % n);
  uint64_t last = k0 + (count - 1);
  for (;;) {
    if (k >= k0) emit(ctx, k, m);
    if (k == last) break;
    ++k;
    s = oracle_lcg_next(s);
    if ((k & (BLOCK - 1)) == 0)
      m = (uint64_t)(((u128)m0 + oracle_block_seed(s0, k >> ORACLE_BLOCK_LOG2)) % n);
    else
      m = (uint64_t)(((u128)m + s) % n);
  }
  return 0;
}

struct gen_ctx {
  uint64_t n, e, k0;
  uint64_t* c;
  double* r;
  uint64_t* m;
  oracle_stats* st;
};

static void emit_gen(void* vp, uint64_t k, uint64_t m) {
  struct gen_ctx* g = (struct gen_ctx*)vp;
  uint64_t c = oracle_powmod(m, g->e, g->n);
  if (g->c) g->c[k - g->k0] = c;
  if (g->r) g->r[k - g->k0] = oracle_ratio(c, g->n);
}

static void emit_msg(void* vp, uint64_t k, uint64_t m) {
  struct gen_ctx* g = (struct gen_ctx*)vp;
  g->m[k - g->k0] = m;
}

int oracle_generate(uint64_t p, uint64_t q, uint64_t e, uint64_t m0, uint64_t s0, uint64_t k0,
                    uint64_t count, uint64_t* c_out, double* r_out) {
  int rc = instance_ok(p, q, e, m0, s0);
  if (rc) return rc;
  struct gen_ctx g = {p * q, e, k0, c_out, r_out, NULL, NULL};
  return walk(p, q, m0, s0, k0, count, emit_gen, &g);
}

int oracle_messages(uint64_t p, uint64_t q, uint64_t m0, uint64_t s0, uint64_t k0, uint64_t count,
                    uint64_t* m_out) {
  int rc = instance_ok(p, q, 1, m0, s0);
  if (rc) return rc;
  struct gen_ctx g = {p * q, 1, k0, NULL, NULL, m_out, NULL};
  return walk(p, q, m0, s0, k0, count, emit_msg, &g);
}

/* ---- algorithm (1): the paper's own CRT formulation ----
 *
 * An independent route to the same outputs inside block 0, used as a pin of
 * the definition above: the message is never formed as one 64-bit number.
 * Its residues modulo p and q are carried instead (Number Theory section,
 * eqs. CRTimplementation), the skip comes from Schrage's decomposition of
 * a s mod Q (Implementation section), each residue is raised to e modulo its
 * own prime, and the ciphertext is the unique value mod n = p q with those
 * residues (Chinese remainder theorem, by Garner's form). */

struct crt_ctx {
  uint64_t p, q;
  uint64_t q_inv_p; /* q^-1 mod p */
};

/* x^e mod m for m < 2^32 (products fit 64 bits). */
static uint64_t pow_small(uint64_t x, uint64_t e, uint64_t m) {
  uint64_t acc = 1 % m;
  for (int b = 63; b >= 0; --b) {
    acc = acc * acc % m;
    if ((e >> b) & 1) acc = acc * (x % m) % m;
  }
  return acc;
}

/* The value x in [0, p q) with x = a (mod p) and x = b (mod q): x = b + q t
 * where t = (a - b) q^-1 mod p. */
static uint64_t crt_value(const struct crt_ctx* k, uint64_t a, uint64_t b) {
  uint64_t d = (a % k->p + k->p - b % k->p) % k->p;
  uint64_t t = d * k->q_inv_p % k->p;
  return b + t * k->q;
}

int oracle_paper_algorithm1(uint64_t p, uint64_t q, uint64_t e, uint64_t m0, uint64_t s0,
                            uint64_t count, uint64_t* c_out, double* r_out) {
  int rc = instance_ok(p, q, e, m0, s0);
  if (rc) return rc;
  const struct crt_ctx k = {p, q, oracle_inverse(q % p, p)};
  uint64_t res[2] = {m0 % p, m0 % q}; /* the message's residues */
  const uint64_t mod[2] = {p, q};
  uint64_t skip = s0;
  for (uint64_t i = 0; i < count; ++i) {
    skip = oracle_lcg_next_schrage(skip);
    uint64_t enc[2];
    for (int j = 0; j < 2; ++j) {
      res[j] = (res[j] + skip % mod[j]) % mod[j];
      enc[j] = pow_small(res[j], e, mod[j]);
    }
    const uint64_t c = crt_value(&k, enc[0], enc[1]);
    if (c_out) c_out[i] = c;
    if (r_out) r_out[i] = oracle_ratio(c, p * q);
  }
  return 0;
}

void oracle_encrypt_array(uint64_t n, uint64_t e, const uint64_t* m, uint64_t* c, uint64_t count) {
  for (uint64_t i = 0; i < count; ++i) c[i] = oracle_powmod(m[i], e, n);
}

/* ---- statistics ---- */

static void stats_add(oracle_stats* st, double r) {
  st->hist[(int)(r * 1024.0)]++;
  if (r < 0.5) st->lt_half++;
  if (r > 0.0) {
    double v = ldexp(r, 128); /* exact: a power-of-two scaling */
    u128 x = (u128)v;         /* r >= 2^-75 makes v an integer below 2^128 */
    u128 lo = ((u128)st->sum_fx[1] << 64) | st->sum_fx[0];
    u128 nlo = lo + x;
    if (nlo < lo) st->sum_fx[2]++;
    st->sum_fx[0] = (uint64_t)nlo;
    st->sum_fx[1] = (uint64_t)(nlo >> 64);
  }
}

void oracle_stats_of(const double* r, uint64_t count, oracle_stats* st) {
  memset(st, 0, sizeof(*st));
  for (uint64_t i = 0; i < count; ++i) stats_add(st, r[i]);
}

static void emit_stats(void* vp, uint64_t k, uint64_t m) {
  struct gen_ctx* g = (struct gen_ctx*)vp;
  (void)k;
  stats_add(g->st, oracle_ratio(oracle_powmod(m, g->e, g->n), g->n));
}

int oracle_consume(uint64_t p, uint64_t q, uint64_t e, uint64_t m0, uint64_t s0, uint64_t k0,
                   uint64_t count, oracle_stats* st) {
  int rc = instance_ok(p, q, e, m0, s0);
  if (rc) return rc;
  memset(st, 0, sizeof(*st));
  struct gen_ctx g = {p * q, e, k0, NULL, NULL, NULL, st};
  return walk(p, q, m0, s0, k0, count, emit_stats, &g);
}

/* ------------------------------------------------------------------------
 * Parameter generation (Implementation section: 32-bit primes, and the safe
 * primes p = 2 p' + 1 with p' prime that the paper recommends).
 * ---------------------------------------------------------------------- */

/* Number of primes (safe primes when safe != 0) in [lo, hi), hi <= 2^32, by a
 * sieve of Eratosthenes over segments: every composite below 2^32 has a prime
 * factor below 2^16.  For safe primes both p and (p - 1)/2 are looked up in
 * sieved segments. */
static void sieve_segment(uint64_t lo, uint64_t len, const uint32_t* small, int ns,
                          unsigned char* isp) {
  memset(isp, 1, len);
  for (uint64_t i = 0; i < len; ++i)
    if (lo + i < 2) isp[i] = 0;
  for (int k = 0; k < ns; ++k) {
    const uint64_t p = small[k];
    if (p * p >= lo + len) break;
    uint64_t m = (lo + p - 1) / p * p;
    if (m < p * p) m = p * p;
    for (; m < lo + len; m += p) isp[m - lo] = 0;
  }
}

static int small_primes(uint32_t* out) {
  static unsigned char comp[1 << 16];
  int ns = 0;
  memset(comp, 0, sizeof(comp));
  for (uint32_t i = 2; i < (1u << 16); ++i) {
    if (comp[i]) continue;
    out[ns++] = i;
    for (uint32_t j = i * i; j < (1u << 16); j += i) comp[j] = 1;
  }
  return ns;
}

uint64_t oracle_count_primes(uint64_t lo, uint64_t hi, int safe) {
  if (hi > (1ULL << 32)) hi = 1ULL << 32;
  if (lo >= hi) return 0;
  static uint32_t small[6542];
  const int ns = small_primes(small);
  const uint64_t SEG = 1ULL << 22;
  unsigned char* a = (unsigned char*)malloc(SEG);
  unsigned char* b = (unsigned char*)malloc(SEG / 2 + 2);
  uint64_t count = 0;
  for (uint64_t s = lo; s < hi; s += SEG) {
    const uint64_t len = hi - s < SEG ? hi - s : SEG;
    sieve_segment(s, len, small, ns, a);
    if (!safe) {
      for (uint64_t i = 0; i < len; ++i) count += a[i];
      continue;
    }
    /* halves (p - 1)/2 of the candidates p in [s, s + len) lie in [h0, h0 + hl) */
    const uint64_t h0 = s / 2 > 0 ? (s - 1) / 2 : 0;
    const uint64_t hl = (s + len - 1) / 2 - h0 + 1;
    sieve_segment(h0, hl, small, ns, b);
    for (uint64_t i = 0; i < len; ++i) {
      const uint64_t p = s + i;
      if (a[i] && p >= 5 && b[(p - 1) / 2 - h0]) ++count;
    }
  }
  free(a);
  free(b);
  return count;
}

/* Smallest p >= x, p < 2^32, prime (safe if asked) with p mod f != 1 for each
 * f in exps[0..nexp); 0 if there is none. */
uint64_t oracle_next_prime(uint64_t x, int safe, const uint32_t* exps, int nexp) {
  for (uint64_t p = x; p < (1ULL << 32); ++p) {
    int ok = oracle_is_prime(p) && (!safe || (p >= 5 && oracle_is_prime((p - 1) / 2)));
    for (int f = 0; ok && f < nexp; ++f)
      if (p % exps[f] == 1) ok = 0;
    if (ok) return p;
  }
  return 0;
}

/* ------------------------------------------------------------------------
 * Statistical battery (Tests section), counted from the oracle's own
 * outputs by the definitions stated in oracle.h.
 * ---------------------------------------------------------------------- */
static uint32_t bin_of(double r, double b, uint32_t nb) {
  uint32_t x = (uint32_t)(r * b);
  return x < nb ? x : nb - 1;
}

int oracle_battery_add(uint64_t p, uint64_t q, uint64_t e, uint64_t m0, uint64_t s0, uint64_t k0,
                       uint64_t count, oracle_battery* B) {
  if (count == 0) return 0;
  double* r = (double*)malloc(count * sizeof(double));
  if (!r) return -9;
  int rc = oracle_generate(p, q, e, m0, s0, k0, count, NULL, r);
  if (rc == 0) rc = oracle_battery_values(r, k0, count, B);
  free(r);
  return rc;
}

int oracle_battery_values(const double* r, uint64_t k0, uint64_t count, oracle_battery* B) {
  if (count == 0) return 0;
  const uint64_t last = k0 + (count - 1);
  for (uint64_t i = 0; i < count; ++i) B->freq[bin_of(r[i], 1048576.0, 1u << 20)]++;
  B->outputs += count;
  /* aligned blocks of 8 indices inside [k0, last] */
  for (uint64_t k8 = (k0 + 7) / 8 * 8; k8 >= k0 && k8 <= last && last - k8 >= 7; k8 += 8) {
    const double* x = r + (k8 - k0);
    for (int t = 0; t < 4; ++t)
      B->serial2[bin_of(x[2 * t], 1024.0, 1024) * 1024 + bin_of(x[2 * t + 1], 1024.0, 1024)]++;
    for (int t = 0; t < 2; ++t)
      B->serial3[(bin_of(x[3 * t], 100.0, 100) * 100 + bin_of(x[3 * t + 1], 100.0, 100)) * 100 +
                 bin_of(x[3 * t + 2], 100.0, 100)]++;
    for (int t = 0; t < 2; ++t) {
      uint32_t c = 0;
      for (int j = 0; j < 4; ++j) c = c * 32 + bin_of(x[4 * t + j], 32.0, 32);
      B->serial4[c]++;
    }
    uint32_t c5 = 0, c6 = 0, seen = 0;
    for (int j = 0; j < 5; ++j) c5 = c5 * 16 + bin_of(x[j], 16.0, 16);
    for (int j = 0; j < 6; ++j) c6 = c6 * 10 + bin_of(x[j], 10.0, 10);
    B->serial5[c5]++;
    B->serial6[c6]++;
    /* number of distinct card values among the first five */
    int distinct = 0;
    for (int j = 0; j < 5; ++j) {
      uint32_t v = bin_of(x[j], 16.0, 16);
      if (!(seen & (1u << v))) {
        seen |= 1u << v;
        ++distinct;
      }
    }
    B->poker[distinct]++;
    if (k8 > UINT64_MAX - 8) break;
  }
  /* aligned blocks of 32: the maximum M, binned by floor(1024 M^32) */
  for (uint64_t k32 = (k0 + 31) / 32 * 32; k32 >= k0 && k32 <= last && last - k32 >= 31; k32 += 32) {
    double mx = 0.0;
    for (int j = 0; j < 32; ++j) {
      double v = r[k32 - k0 + j];
      if (v > mx) mx = v;
    }
    double t = mx;
    for (int j = 0; j < 5; ++j) t = t * t;
    B->maxt[bin_of(t, 1024.0, 1024)]++;
    if (k32 > UINT64_MAX - 32) break;
  }
  /* aligned blocks of 64: the run that starts at the block's first index */
  for (uint64_t k64 = (k0 + 63) / 64 * 64; k64 >= k0 && k64 <= last && last - k64 >= 63; k64 += 64) {
    const double* x = r + (k64 - k0);
    const int b = x[0] > 0.5;
    int len = 1;
    while (len < 64 && (x[len] > 0.5) == b) ++len;
    B->runs[b][len - 1]++;
    if (k64 > UINT64_MAX - 64) break;
  }
  /* aligned blocks of 2^14: balls in 2^20 urns, collisions = balls - distinct urns */
  const uint64_t T = 1u << 14;
  uint64_t kt = (k0 + T - 1) / T * T;
  if (kt >= k0 && kt <= last && last - kt >= T - 1) {
    uint32_t* urn = (uint32_t*)calloc(1u << 15, sizeof(uint32_t));
    if (!urn) return -9;
    for (; kt >= k0 && kt <= last && last - kt >= T - 1; kt += T) {
      uint32_t distinct = 0;
      for (uint64_t j = 0; j < T; ++j) {
        const uint32_t u = bin_of(r[kt - k0 + j], 1048576.0, 1u << 20);
        if (!(urn[u >> 5] & (1u << (u & 31)))) {
          urn[u >> 5] |= 1u << (u & 31);
          ++distinct;
        }
      }
      const uint32_t c = (uint32_t)T - distinct;
      B->coll[c < 255 ? c : 255]++;
      for (uint64_t j = 0; j < T; ++j) {
        const uint32_t u = bin_of(r[kt - k0 + j], 1048576.0, 1u << 20);
        urn[u >> 5] = 0;
      }
      if (kt > UINT64_MAX - T) break;
    }
    free(urn);
  }
  /* leading bits of 20 successive values: trials j = 0, 1, 2 of each block of
   * 2^20 indices, 2^14 balls of 20 indices each from the block's start */
  const uint64_t BALL = 20, TRIAL = BALL << 14, BLOCK = 1ULL << 20;
  uint32_t* urn2 = NULL;
  for (uint64_t blk = k0 & ~(BLOCK - 1);; blk += BLOCK) {
    for (uint64_t j = 0; j < 3; ++j) {
      const uint64_t ts = blk + j * TRIAL;
      if (ts < k0 || ts > last || last - ts < TRIAL - 1) continue;
      if (!urn2 && !(urn2 = (uint32_t*)calloc(1u << 15, sizeof(uint32_t)))) return -9;
      uint32_t distinct = 0;
      for (uint64_t g = 0; g < (1u << 14); ++g) {
        uint32_t u = 0;
        for (uint64_t i = 0; i < BALL; ++i)
          u |= (uint32_t)(r[ts - k0 + g * BALL + i] * 2.0) << i;
        if (!(urn2[u >> 5] & (1u << (u & 31)))) {
          urn2[u >> 5] |= 1u << (u & 31);
          ++distinct;
        }
      }
      const uint32_t c = (1u << 14) - distinct;
      B->coll_msb[c < 255 ? c : 255]++;
      memset(urn2, 0, (1u << 15) * sizeof(uint32_t));
    }
    if (blk >= (last & ~(BLOCK - 1))) break;
  }
  free(urn2);
  return 0;
}
