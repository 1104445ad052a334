/*
 * rsaprng.h -- C ABI of the MI355X (gfx950) implementation of the
 * non-cryptographic RSA-exponentiation pseudorandom generator of
 * Datephanyawat & Beale (arXiv:1811.11629).
 *
 * The generator (paper: Introduction eq. encrypt2, Pseudorandom skips,
 * Implementation algorithm (1)):
 *   skips     s_j = s0 * a^j mod Q,  Q = 2^63 - 25, a = 2307085864
 *   messages  m_k = (m_{k-1} + s_k) mod n inside each block of 2^20 indices;
 *             at a block start bB the message is re-seeded to
 *             (m0 + (s_1 + ... + s_bB mod Q)) mod n, which makes every index
 *             reachable by a jump (the paper's closed form, eq. pseudoskip,
 *             is evaluated exactly for the skips; the re-seeding is this
 *             library's reading of how to jump the message sum)
 *   outputs   c_k = m_k^e mod n   (n = p q, p and q 32-bit primes, e small odd)
 *             r_k = RN(RN(c_k) / RN(n)) in IEEE binary64, with 1 - 2^-53
 *             returned where that quotient rounds to 1.0 (the guard the paper
 *             asks for after algorithm (1)).
 * Every output is a pure function of (p, q, e, m0, s0, k): it does not depend
 * on streams, tiling, batch composition, kernel variant or device.
 *
 * Conventions
 *  - Functions returning int return RSAPRNG_OK (0) or a negative status.
 *  - Output buffers and stats records are DEVICE pointers owned by the caller,
 *    8-byte aligned; any output pointer may be NULL to skip that output.
 *  - Streams are hipStream_t values passed as void* (NULL = default stream).
 *  - Generation calls only enqueue work on the stream.  Launch errors return
 *    RSAPRNG_E_HIP; a fault is reported when the caller synchronises.  A
 *    kernel-detected error (a bounded wait that expired) is returned by the
 *    next rsaprng_check_device_error() on the same stream.
 *  - Handles are immutable after creation and may be shared by threads; each
 *    stream gets its own launch scratch, so concurrent launches must use
 *    different streams (launches on one stream are ordered).
 *  - No function here allocates on the hot path except where stated
 *    (first use of a stream grows its scratch; batch/server creation).
 */
#ifndef RSAPRNG_H
#define RSAPRNG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define RSAPRNG_BLOCK_LOG2 20                 /* output-defining: block of the re-seeding */
#define RSAPRNG_Q 9223372036854775783ULL      /* skip modulus 2^63 - 25 (Implementation) */
#define RSAPRNG_A 2307085864ULL               /* skip multiplier, a primitive root mod Q */

enum rsaprng_status {
  RSAPRNG_OK = 0,
  RSAPRNG_E_NOT_PRIME = -1,      /* p or q fails deterministic Miller-Rabin */
  RSAPRNG_E_EQUAL_PRIMES = -2,   /* p == q */
  RSAPRNG_E_PRIME_RANGE = -3,    /* p or q outside [2^31, 2^32) */
  RSAPRNG_E_BAD_EXPONENT = -4,   /* e == 0 or gcd(e, lambda(n)) != 1 (covers even e) */
  RSAPRNG_E_BAD_SEED = -5,       /* create_ex: m0 >= n, or s0 not in [1, Q-1] */
  RSAPRNG_E_RANGE = -6,          /* k0 + count > 2^64, or a launch larger than 2^32 tiles */
  RSAPRNG_E_NULL = -7,           /* required pointer is NULL */
  RSAPRNG_E_ALIGN = -8,          /* device pointer not 8-byte aligned */
  RSAPRNG_E_OOM = -9,            /* device or host allocation failed */
  RSAPRNG_E_HIP = -10,           /* a HIP runtime call failed */
  RSAPRNG_E_BUSY = -11,          /* server: arena full or queue full */
  RSAPRNG_E_ARG = -12,           /* other invalid argument */
  RSAPRNG_E_DEVICE = -13,        /* a kernel reported an error (bounded wait expired) */
  RSAPRNG_E_NO_DEVICE = -14,     /* no usable gfx950 device */
  RSAPRNG_E_TOO_LARGE = -15      /* rsaprng_pool_generate_noalloc: the launch does not fit
                                    its fixed scratch */
};

/* ---------------------------------------------------------------------------
 * Instance parameters (host only; no device needed).
 * rsaprng_params_init validates (p, q, e) by the paper's rules -- both 32-bit
 * primes by deterministic Miller-Rabin (five bases below 2^32, Implementation
 * section), p != q, gcd(e, lambda(n)) = 1 so the decryption exponent exists
 * (Number Theory, eq. RSAd) -- and fills the per-instance constants the
 * kernels use.  Returns a status; *out is written only on success.
 * ------------------------------------------------------------------------ */
typedef struct {
  uint64_t n;        /* p q */
  uint64_t m0;       /* message seed, < n */
  uint64_t s0;       /* skip seed, in [1, Q-1] */
  uint64_t ce;       /* R^e mod n, R = 2^64 (Montgomery correction) */
  uint32_t ninv;     /* -n^-1 mod 2^32 */
  uint32_t e, p, q;
  double nd;         /* RN(n) */
  double pd, qd;     /* p, q */
  double pinv, qinv; /* RN(1/p), RN(1/q) */
  double qinvp;      /* q^-1 mod p (Garner's constant, Number Theory section) */
  double kp, kq;     /* 2^32 mod p, 2^32 mod q */
  double nrcp;       /* RN(1 / RN(n)) */
  uint32_t ep, eq;   /* exponents applied mod p and mod q: both e for an ordinary
                        instance; see rsaprng_pool_create_dual (e is then 0) */
  /* Split forms of the CRT variant's constants.  For K = 2^32 mod p:
   * kp_hi = K - (K mod 2^17), kp_lo = K mod 2^17, kp_quo = RN(K RN(1/p)); the
   * kernels reduce H K mod p for integers |H| < 2^35 as
   * fma(H, kp_lo, fma(-rint(H kp_quo), p, H kp_hi)), every step exact.  The same
   * for 2^32 mod q (kq_*) and for Garner's q^-1 mod p (gp_*). */
  double kp_lo, kp_hi, kp_quo;
  double kq_lo, kq_hi, kq_quo;
  double gp_lo, gp_hi, gp_quo;
  double nrcp_lo;    /* RN(RN(1 - nd nrcp) nrcp): nrcp + nrcp_lo = 1/nd to ~2^-105 */
} rsaprng_params;    /* 208 bytes; the device-side instance record */

int rsaprng_params_init(uint64_t p, uint64_t q, uint64_t e, uint64_t m0, uint64_t s0,
                        rsaprng_params* out);

/* Deterministic Miller-Rabin for any 64-bit n (twelve bases), as the library
 * uses it for validation.  Host only. */
int rsaprng_is_prime(uint64_t n);

/* s0 * a^k mod Q and the block seed (s_1 + ... + s_{bB}) mod Q, B = 2^20, as
 * the host library computes them (eqs. congruentialgenerator1, pseudoskip).
 * Host only; exposed for tests. */
uint64_t rsaprng_skip_at(uint64_t s0, uint64_t k);
uint64_t rsaprng_block_seed(uint64_t s0, uint64_t b);

/* ---------------------------------------------------------------------------
 * Single instances.
 * rsaprng_create: m0 = seed mod n, s0 = 1.  rsaprng_create_ex sets both.
 * Return NULL on error; rsaprng_last_error() (thread-local) gives the status.
 * rsaprng_destroy: the caller must have synchronised streams that use h.
 * ------------------------------------------------------------------------ */
typedef struct rsaprng_s* rsaprng_t;
rsaprng_t rsaprng_create(uint64_t p, uint64_t q, uint64_t e, uint64_t seed);
rsaprng_t rsaprng_create_ex(uint64_t p, uint64_t q, uint64_t e, uint64_t m0, uint64_t s0);
int rsaprng_last_error(void);
const char* rsaprng_strerror(int code);
void rsaprng_destroy(rsaprng_t h);
int rsaprng_get_params(rsaprng_t h, rsaprng_params* out);

/* out_u64[j] = c_{k0+j}, out_f64[j] = r_{k0+j} for j < count (eqs. encrypt2
 * and CodeFloatingPointStep).  count == 0 is a no-op.  k0 + count <= 2^64. */
int rsaprng_generate(rsaprng_t h, uint64_t k0, uint64_t count, uint64_t* out_u64,
                     double* out_f64, void* stream);

/* Vector mode (Parallelization section, eq. vectorize and the stream splitting
 * after it): the instance split into M_v = mv substreams advanced together.
 * Substream g (0 <= g < mv) is the instance's sequence with the skip seed
 * s0 a^(g J) mod Q, J = floor((Q-1)/mv), and the same message seed m0 (the
 * paper leaves the message starts open; this is the library's reading).  The
 * t-th vector call (t = 1, 2, ...) returns element g = the output of substream
 * g after t updates, i.e. its index k = t (so the first call never returns the
 * seed itself).  Flattened, f = (t - 1) mv + g, and this writes
 * out_u64[j] = c and out_f64[j] = r of f = f0 + j for j < count; either
 * pointer may be NULL.  Any f0 is allowed: a range starting inside a 2^20
 * block walks every substream from the block start (mv (t mod 2^20) skip
 * steps of lead-in).  variant: 0 auto (CRT), 1 Montgomery-64, 2 CRT, as in
 * rsaprng_config; the outputs do not depend on it.
 * Limits: 1 <= mv <= RSAPRNG_VECTOR_MAX_MV, count <= RSAPRNG_VECTOR_MAX_COUNT,
 * f0 + count <= RSAPRNG_VECTOR_MAX_END (else RSAPRNG_E_ARG / RSAPRNG_E_RANGE).
 * Enqueued on `stream`; grows the stream's scratch to at most 8 (2^26 + 4 ng)
 * bytes, ng = min(mv, count) (about 16 MB when mv << 2^21). */
#define RSAPRNG_VECTOR_MAX_MV (1ULL << 24)
#define RSAPRNG_VECTOR_MAX_COUNT (1ULL << 56)
#define RSAPRNG_VECTOR_MAX_END (1ULL << 62)
int rsaprng_generate_vector(rsaprng_t h, uint64_t mv, uint64_t f0, uint64_t count,
                            uint64_t* out_u64, double* out_f64, int variant, void* stream);

/* Many instances in one launch: request i writes c_{k0+j}, r_{k0+j} of reqs[i].h
 * to out_u64[out_off + j], out_f64[out_off + j].  reqs is a host array. */
typedef struct {
  rsaprng_t h;
  uint64_t k0, count, out_off;
} rsaprng_req;
int rsaprng_generate_batch(const rsaprng_req* reqs, size_t nreq, uint64_t* out_u64,
                           double* out_f64, void* stream);

/* ---------------------------------------------------------------------------
 * Fused consume (statistics instead of stores).
 * Over k in [k0, k0+count): the exact sum of r_k as a 192-bit fixed-point
 * number with LSB 2^-128 (every r_k is a multiple of 2^-116, so the sum is
 * exact and independent of order), the count of r_k < 0.5, and the 1024-bin
 * histogram hist[floor(1024 r_k)] -- the paper's one-dimensional frequency
 * and half-split statistics (Tests section).  *out is a DEVICE record; it is
 * overwritten (not accumulated).
 * ------------------------------------------------------------------------ */
typedef struct {
  uint64_t sum_fx[3];   /* normalised exact sum, little-endian limbs, LSB 2^-128 */
  uint64_t lt_half;     /* number of r_k < 0.5 */
  uint64_t count;       /* number of outputs reduced */
  double sum;           /* the exact sum rounded once to binary64 */
  uint64_t acc32[6];    /* not a result: the kernels' exact accumulator (work-groups add
                           32-bit digit sums here with device atomics; the finalisation
                           normalises them into sum_fx and sum), kept in the record so a
                           consume launch needs no scratch of its own */
  uint64_t hist[1024];
} rsaprng_stats;
int rsaprng_consume(rsaprng_t h, uint64_t k0, uint64_t count, rsaprng_stats* out_dev,
                    void* stream);

/* ---------------------------------------------------------------------------
 * Pools: device-resident tables of many instances (the paper's
 * parameterisation, one modulus per stream: Parallelization section).
 * seed[i] gives m0 = seed mod n; s0 may be NULL (all 1).  On error returns NULL
 * and sets rsaprng_last_error(); err_index (may be NULL) receives the first
 * bad instance.
 * ------------------------------------------------------------------------ */
typedef struct rsaprng_pool_s* rsaprng_pool_t;
rsaprng_pool_t rsaprng_pool_create(size_t n, const uint64_t* p, const uint64_t* q,
                                   const uint64_t* e, const uint64_t* seed, const uint64_t* s0,
                                   size_t* err_index);
/* Instances with different small exponents mod p and mod q (the footnote on
 * CRT exponents): c_p = m_p^ep mod p, c_q = m_q^eq mod q, recombined by Garner,
 * which is m^e mod n for the large exponent e with e = ep mod (p-1) and
 * e = eq mod (q-1) (rsaprng_dual_exponent).  Requires gcd(ep, p-1) = 1,
 * gcd(eq, q-1) = 1 and ep = eq mod gcd(p-1, q-1) (so that e exists; always
 * true for safe primes and odd exponents).  Launches over such a pool use the
 * CRT variant whatever the configuration asks. */
rsaprng_pool_t rsaprng_pool_create_dual(size_t n, const uint64_t* p, const uint64_t* q,
                                        const uint64_t* ep, const uint64_t* eq,
                                        const uint64_t* seed, const uint64_t* s0,
                                        size_t* err_index);
/* The record of one dual-exponent instance, validated as for the pool (host
 * only; *out written on success). */
int rsaprng_params_init_dual(uint64_t p, uint64_t q, uint64_t ep, uint64_t eq, uint64_t m0,
                             uint64_t s0, rsaprng_params* out);
/* The combined exponent: the smallest e >= 1 with e = ep mod (p-1) and
 * e = eq mod (q-1).  Host only; RSAPRNG_E_BAD_EXPONENT if there is none. */
int rsaprng_dual_exponent(uint64_t p, uint64_t q, uint64_t ep, uint64_t eq, uint64_t* e);
void rsaprng_pool_destroy(rsaprng_pool_t pool);
size_t rsaprng_pool_size(rsaprng_pool_t pool);

typedef struct {
  uint32_t inst;        /* pool index */
  uint32_t reserved;
  uint64_t k0, count;
  uint64_t out_off;     /* generate: output element offset; consume: stats record index */
} rsaprng_pool_req;

/* Kernel configuration.  Outputs never depend on it.
 * Environment variables read by the library (performance and diagnostics only):
 *   RSAPRNG_VARIANT          variant taken when variant is 0 (default 2, CRT)
 *   RSAPRNG_PREFIX           prefix form taken when prefix is not 0, 1 or 2
 *                            (default 0, two passes)
 *   RSAPRNG_SPIN_LIMIT       polls of a look-back word before the one-pass kernel
 *                            reports RSAPRNG_E_DEVICE (default 2^22)
 *   RSAPRNG_CLASS_MIN_TILES  in a two-pass launch with 16 indices per lane, the
 *                            fewest tiles an exponent class takes a launch of its
 *                            own for (default 16384)
 *   RSAPRNG_TUNE_LOG         set: the autotuner prints each trial to stderr */
typedef struct {
  int variant;          /* 0 auto, 1 Montgomery-64 integer path, 2 CRT with binary64 residues */
  int lanes_per_tile;   /* work-group size: 0 default, else 256 or 512 */
  int per_lane;         /* consecutive indices per lane: 0 default, else 8 or 16 (two
                           passes: 16 with 256 lanes and 2 chunks per wave for CRT
                           generate launches, one tile launch per exponent class;
                           other launches take 4 chunks of 8, the same tile) */
  int persistent;       /* 1: grid of resident work-groups looping over the tiles */
  int wg_per_cu;        /* persistent grid size per compute unit (0 = default) */
  int order;            /* 0 request order, 1 longest-first by exponent cost */
  int prefix;           /* 0 two passes (tile sums, scan, generate); 1 one pass with a
                           decoupled look-back over the preceding tiles; 2 chain-serial:
                           one work-group walks each chain (a request's indices inside
                           one 2^20 block) in order, carrying the message prefix */
  int chunks_per_wave;  /* two passes and chain-serial: 64*per_lane chunks per wave per tile
                           (1 for chain-serial with per_lane 16, which runs as such for
                           CRT launches whose instances all share one exponent: e = 3 in
                           generate mode, 3, 5, 7, 17, 257 or 65537 in consume mode with
                           256 lanes; other launches take two chunks of 8 indices per
                           lane, the same tile) */
} rsaprng_config;

/* One-shot batched launches over a pool (reqs is a host array). */
int rsaprng_pool_generate(rsaprng_pool_t pool, const rsaprng_pool_req* reqs, size_t nreq,
                          uint64_t* out_u64, double* out_f64, const rsaprng_config* cfg,
                          void* stream);
int rsaprng_pool_consume(rsaprng_pool_t pool, const rsaprng_pool_req* reqs, size_t nreq,
                         rsaprng_stats* stats_dev, const rsaprng_config* cfg, void* stream);

/* rsaprng_pool_generate without any allocation, for callers that cannot
 * allocate device memory: code that runs under stream capture, tight serving
 * loops, harnesses that forbid hipMalloc.  Same arguments, outputs and status
 * codes as rsaprng_pool_generate (the outputs are identical), except:
 *  - all launch scratch lives in one fixed array of RSAPRNG_NOALLOC_SCRATCH_BYTES
 *    of device memory per GPU, taken once per device by the library and held
 *    until the process ends; the chain plan is staged in fixed host arrays.
 *    Nothing is allocated on the device or the host by the call;
 *  - a launch must fit that scratch: at most RSAPRNG_NOALLOC_MAX_CHAINS chains
 *    (one per request and 2^20 block it touches, after merging requests that
 *    continue each other, plus for the chain-serial form one per request that
 *    starts beyond the first tile of its block), and its tile arrays (12 bytes
 *    per tile plus 16 per
 *    wave chunk of 64 * per_lane indices) within the rest; otherwise
 *    RSAPRNG_E_TOO_LARGE and nothing is enqueued.  With the default tile of
 *    2048 indices that is about 2^29 outputs per call;
 *  - the one-pass form (prefix 1) is replaced by two passes (prefix 0);
 *  - the pool must belong to the current device (RSAPRNG_E_ARG otherwise), and
 *    devices 0..7 only (RSAPRNG_E_NO_DEVICE).
 * Every call on a GPU shares that GPU's scratch, which keeps the last call's
 * contents: calls on one stream are ordered, but calls that overlap on one GPU
 * (on different streams without an ordering between them) race and may
 * corrupt each other's outputs.  Returns before the launch completes, like
 * rsaprng_pool_generate; a later call on a different stream first waits for
 * the launch that last used the same upload slot. */
#define RSAPRNG_NOALLOC_SCRATCH_BYTES (32u << 20)
#define RSAPRNG_NOALLOC_MAX_CHAINS 16384
int rsaprng_pool_generate_noalloc(rsaprng_pool_t pool, const rsaprng_pool_req* reqs, size_t nreq,
                                  uint64_t* out_u64, double* out_f64, const rsaprng_config* cfg,
                                  void* stream);

/* Prepared batches: the request table and tile plan are uploaded once and the
 * launch (queue reset + persistent kernel) is captured in a hipGraph on the
 * given stream; rsaprng_batch_run replays it.  Outputs go to the buffers given
 * at creation.  mode 0 = generate (out_u64/out_f64), 1 = consume (stats_dev). */
typedef struct rsaprng_batch_s* rsaprng_batch_t;
int rsaprng_batch_create(rsaprng_pool_t pool, const rsaprng_pool_req* reqs, size_t nreq, int mode,
                         uint64_t* out_u64, double* out_f64, rsaprng_stats* stats_dev,
                         const rsaprng_config* cfg, void* stream, rsaprng_batch_t* out);
int rsaprng_batch_run(rsaprng_batch_t b, void* stream);
/* RSAPRNG_E_DEVICE if a replay flagged an error since the last call (the caller
 * must have synchronised the stream of the replays), else RSAPRNG_OK. */
int rsaprng_batch_check(rsaprng_batch_t b);
/* The same launch enqueued without its graph, with HIP events recorded on
 * `stream` between its kernels: per-kernel durations without a profiler. */
int rsaprng_batch_run_timed(rsaprng_batch_t b, void* stream);
/* Average durations in ms over the timed runs since the previous call: ms[0]
 * chain setup (with statistics zeroing), ms[1] prefix pass(es), ms[2] tile
 * kernel, ms[3] statistics finalisation; *runs (may be NULL) receives their
 * number.  Waits for those runs, then forgets them. */
int rsaprng_batch_kernel_ms(rsaprng_batch_t b, double* ms, int* runs);
void rsaprng_batch_destroy(rsaprng_batch_t b);

/* Autotuner: times every kernel configuration in its search space on this
 * request set, checks that all of them produce byte-identical outputs, and
 * writes the fastest to *best (and its time per launch in ms to *best_ms).
 * Generate mode overwrites out_u64 / out_f64 over [0, max(out_off + count)):
 * before each configuration's run both are filled with a sentinel, so an
 * output a configuration failed to write would change the comparison; on
 * return the requested elements hold the outputs and any element between them
 * the sentinel 0xA5A5A5A5A5A5A5A5.  Consume mode overwrites the records.
 * If cache_path is non-NULL the result is stored there (JSON lines keyed by a
 * signature of the library build, the device and the workload: exponent mix,
 * request count and total outputs) and reused on the next call with the same
 * signature. */
int rsaprng_autotune(rsaprng_pool_t pool, const rsaprng_pool_req* reqs, size_t nreq, int mode,
                     uint64_t* out_u64, double* out_f64, rsaprng_stats* stats_dev,
                     const char* cache_path, void* stream, rsaprng_config* best, double* best_ms);

/* ---------------------------------------------------------------------------
 * Server: continuous batching over a pool kept resident on the device.
 * Requests are admitted while the output arena (arena_bytes of device memory
 * owned by the server) has room for 16 * count bytes; every iteration launches
 * one batch over the next tiles of all admitted requests, so requests that
 * arrive while others run join at the next iteration.  Completed requests'
 * outputs stay in the arena until released.  A background thread drives the
 * loop; submit/poll/release are thread-safe.
 * ------------------------------------------------------------------------ */
typedef struct rsaprng_server_s* rsaprng_server_t;
typedef struct {
  size_t arena_bytes;         /* device output arena */
  uint64_t iter_outputs;      /* max outputs per iteration (0 = default 2^26) */
  uint64_t chunk_outputs;     /* max outputs of one request per iteration (0 = default 2^22) */
  size_t max_queue;           /* max waiting requests (0 = 1<<20) */
  rsaprng_config cfg;
  int policy;                 /* order of the requests' chunks in an iteration:
                                 RSAPRNG_SRV_ROUND_ROBIN (0) or RSAPRNG_SRV_SHORTEST_FIRST
                                 (fewest outputs left first) */
} rsaprng_server_opts;
#define RSAPRNG_SRV_ROUND_ROBIN 0
#define RSAPRNG_SRV_SHORTEST_FIRST 1
typedef struct {
  uint64_t tag;
  const uint64_t* c;          /* device pointers into the arena */
  const double* r;
  uint64_t count;
  double t_submit, t_admit, t_done;   /* seconds on the server's monotonic clock */
} rsaprng_completion;
int rsaprng_server_create(rsaprng_pool_t pool, const rsaprng_server_opts* opts,
                          rsaprng_server_t* out);
int rsaprng_server_submit(rsaprng_server_t s, uint32_t inst, uint64_t k0, uint64_t count,
                          uint64_t tag);
/* Returns the number of completions written (>= 0) or a status. */
int rsaprng_server_poll(rsaprng_server_t s, rsaprng_completion* out, size_t max);
/* Copies outputs [offset, offset + count) of a completed, unreleased request to
 * dst_u64 / dst_f64 (host or device memory; either may be NULL) and waits for
 * the copy on `stream`.  RSAPRNG_E_ARG if tag is not a completed request. */
int rsaprng_server_read(rsaprng_server_t s, uint64_t tag, uint64_t offset, uint64_t count,
                        uint64_t* dst_u64, double* dst_f64, void* stream);
/* Frees a completed request's arena space; its completion pointers become invalid. */
int rsaprng_server_release(rsaprng_server_t s, uint64_t tag);
double rsaprng_server_now(rsaprng_server_t s);
/* Iterations run, outputs produced, and requests waiting/active, for reports. */
int rsaprng_server_stats(rsaprng_server_t s, uint64_t* iterations, uint64_t* outputs,
                         uint64_t* waiting, uint64_t* active);
/* Open-loop load generator: submits request i (tag 2^63 + i) at t_arrival[i]
 * seconds after the call (non-decreasing), releases each on completion, and
 * returns when all have completed.  t_admit / t_done (may be NULL) receive the
 * times relative to the same origin. */
int rsaprng_server_replay(rsaprng_server_t s, size_t n, const uint32_t* inst, const uint64_t* k0,
                          const uint64_t* count, const double* t_arrival, double* t_admit,
                          double* t_done);
/* Host-only dry run of the server's scheduler, for tests (no device), with the
 * given policy (RSAPRNG_SRV_*).  Request i
 * arrives before iteration arrive_iter[i] (non-decreasing); every iteration
 * completes before the next; a finished request is released hold_iters
 * iterations later.  One record of seven words per planned chunk -- request,
 * iteration, first index, count, arena offset, flags (1 continues from saved
 * state, 2 saves state at its end), state slot -- is written to log while
 * fewer than max_log have been written.  Returns the number of chunks or a status. */
int64_t rsaprng_server_simulate(const rsaprng_config* cfg, uint64_t arena_elems,
                                uint64_t iter_outputs, uint64_t chunk_outputs, int policy,
                                size_t n, const uint64_t* k0, const uint64_t* count,
                                const uint64_t* arrive_iter, uint64_t hold_iters, uint64_t* log,
                                size_t max_log);
void rsaprng_server_destroy(rsaprng_server_t s);

/* ---------------------------------------------------------------------------
 * Statistical battery as a fused consumer (Tests section: one-dimensional
 * frequency with 2^20 bins; serial tests in D = 2..6 dimensions with 2^20 or
 * 10^6 bins; the poker test with five cards of sixteen denominations; the
 * maximum of t = 32).  The counts of every output r_k, k in [k0, k0+count), of
 * every request are accumulated into ONE device record; no output is stored.
 * Grouping (this library's reading; the tuples must not depend on how the work
 * is tiled): tuples are taken inside aligned blocks of 8 indices (k = 8j ..
 * 8j+7, absolute index): D-tuples at offsets 0, D, 2D, ... that fit in the
 * block (floor(8/D) per block), the poker hand is offsets 0..4, and the
 * maximum of 32 uses aligned blocks of 32 indices; a block counts only when
 * all its indices are requested.  Bins: floor(b r) for b bins per coordinate
 * (a serial cell is the mixed-radix number of its coordinates, first index
 * most significant), the poker class is the number of distinct floor(16 r),
 * and the maximum M of 32 goes to bin floor(1024 M^32) (M^32 by five exact
 * squarings; it is uniform when the r are).  Collisions: every aligned block
 * of 2^14 indices is one trial of 2^14 balls thrown into 2^20 urns (urn
 * floor(2^20 r)); C = 2^14 - (number of distinct urns) is counted in coll[C]
 * (C >= 255 in coll[255]).  Gaps (runs of 0s and 1s, b = [r > 1/2]): in every
 * aligned block of 64 indices, the run that starts at the block's first index
 * has value b and length L (1..64, capped by the block): runs[b][L - 1].
 * Collisions of leading bits (the Tests section's second collision test, the
 * most significant bit of twenty successive numbers): inside each block of
 * 2^20 indices (the re-seeding blocks), balls of 20 consecutive indices from
 * the block's start; the urn is the 20-bit number whose bit j is the leading
 * bit floor(2 r) of the ball's j-th value; trials of 2^14 consecutive balls,
 * the block's first three (its last 65536 indices take no ball); a trial
 * whose indices are all requested counts C = 2^14 - (distinct urns) in
 * coll_msb[C] (C >= 255 in coll_msb[255]).
 * Requests are taken one by one: a block or trial that only the union of two
 * requests covers is not counted.
 * Counts are unsigned 32-bit (per bin; wraps after 2^32).
 * ------------------------------------------------------------------------ */
#define RSAPRNG_BAT_TESTS 11  /* frequency, serial D = 2..6, poker, max-of-32, collisions,
                                 gaps, collisions of leading bits */
typedef struct {
  uint64_t outputs;           /* number of r_k consumed: the sum of the requests' counts */
  uint64_t reserved;
  uint32_t freq[1 << 20];     /* bin floor(2^20 r) */
  uint32_t serial2[1 << 20];  /* 1024 bins per coordinate */
  uint32_t serial3[1000000];  /* 100 */
  uint32_t serial4[1 << 20];  /* 32 */
  uint32_t serial5[1 << 20];  /* 16 */
  uint32_t serial6[1000000];  /* 10 */
  uint32_t poker[8];          /* [d] = hands with d distinct values, d = 1..5 */
  uint32_t maxt[1024];        /* bin floor(1024 M^32) */
  uint32_t coll[256];         /* [C] = trials of 2^14 balls with C collisions */
  uint32_t runs[2][64];       /* [b][L - 1] = leading runs of value b and length L */
  uint32_t coll_msb[256];     /* [C] = trials of the leading-bit urns with C collisions */
} rsaprng_battery;

/* Zeroes *rec_dev, then accumulates every request into it (reqs[i].out_off is
 * ignored).  Runs the chain-serial CRT kernel, persistent, whatever cfg asks
 * (its work-group walks each chain in order and holds a trial's 2^20-urn
 * bitmap, 128 KB, in LDS, and two 2^20-bit bitmaps of the leading-bit trials in
 * device memory the library keeps per stream, 256 KB per resident work-group);
 * cfg->lanes_per_tile and cfg->chunks_per_wave select its shape. */
int rsaprng_pool_battery(rsaprng_pool_t pool, const rsaprng_pool_req* reqs, size_t nreq,
                         rsaprng_battery* rec_dev, const rsaprng_config* cfg, void* stream);

/* The same battery over values already in device memory: r_dev[j] stands at
 * index j (the groups are aligned to j), j < count, for instance the flattened
 * output of rsaprng_generate_vector, where the tests then see the substreams
 * interleaved (interstream correlations, Tests section).  Zeroes *rec_dev
 * first; enqueued on `stream`.  r_dev must be 8-byte aligned. */
int rsaprng_battery_values(const double* r_dev, uint64_t count, rsaprng_battery* rec_dev,
                           void* stream);

/* Chi-squared statistic, degrees of freedom and p-value (the upper tail
 * P(X >= chi2) of the chi-squared distribution) of each test, in the order of
 * RSAPRNG_BAT_TESTS, from a HOST copy of a record: uniform expectations for the
 * frequency, serial and max tests; for poker the exact probabilities
 * S(5, d) 16 15 ... (16 - d + 1) / 16^5 (S: Stirling numbers of the second
 * kind), with the classes d = 1, 2 merged; for collisions the exact
 * distribution of C for 2^14 balls in 2^20 urns (occupancy recursion; both
 * collision tests); for gaps P(b, L) = 2^-(L+1) for L < 64 and 2^-64 for L = 64.  Collision and gap
 * classes are merged from the tails until each expects at least 5 counts.
 * Host only. */
typedef struct {
  double chi2[RSAPRNG_BAT_TESTS];
  double dof[RSAPRNG_BAT_TESTS];
  double p[RSAPRNG_BAT_TESTS];
  uint64_t samples[RSAPRNG_BAT_TESTS];  /* tuples, hands or maxima counted */
} rsaprng_battery_result;
int rsaprng_battery_report(const rsaprng_battery* rec_host, rsaprng_battery_result* out);

/* Upper tail of the chi-squared distribution with dof degrees of freedom. */
double rsaprng_chi2_sf(double chi2, double dof);

/* ---------------------------------------------------------------------------
 * Parameter generation on the device (Implementation section: the primes of
 * an instance lie in [2^31, 2^32), deterministic Miller-Rabin with the first
 * five prime bases below 2^32, and safe primes p = 2 p' + 1 with p' prime as
 * the recommended class).
 * rsaprng_prime_count: number of primes (safe primes if safe != 0) in
 *   [lo, hi), hi <= 2^32; waits for the result on `stream` (allocates 8 bytes
 *   of device memory for the call).
 * rsaprng_next_primes: for each of n device values x[i], out[i] = the smallest
 *   p in [x[i], min(x[i] + 2^24, 2^32)) that is prime (safe if asked) with
 *   p mod f != 1 for every f in the host array exps[0..nexp) (nexp <= 8, each
 *   f >= 2: the exponent filter gcd(f, p - 1) = 1 for prime f), or 0 if there
 *   is none.  Device arrays, 8-byte aligned; enqueued on `stream`.
 * ------------------------------------------------------------------------ */
int rsaprng_prime_count(uint64_t lo, uint64_t hi, int safe, uint64_t* count, void* stream);
int rsaprng_next_primes(const uint64_t* x, uint64_t n, int safe, const uint32_t* exps, int nexp,
                        uint64_t* out, void* stream);

/* ---------------------------------------------------------------------------
 * Checks and test entry points.
 * ------------------------------------------------------------------------ */
/* Returns RSAPRNG_E_DEVICE if a kernel on this stream's scratch flagged an
 * error since the last call (synchronises the stream), else RSAPRNG_OK. */
int rsaprng_check_device_error(void* stream);

/* c[i] = m[i]^e mod n (and r[i]) for any odd primes p != q below 2^32 with
 * gcd(e, lambda) = 1, using the chosen variant's exponentiation; m, c, r are
 * device arrays (c or r may be NULL).  For bijection checks with small primes. */
int rsaprng_debug_encrypt(uint64_t p, uint64_t q, uint64_t e, int variant, const uint64_t* m,
                          uint64_t* c, double* r, uint64_t count, void* stream);

/* ---------------------------------------------------------------------------
 * Throughput probes (measurement only; nothing is generated).  The roofline
 * figures of the benchmark compare the generator's kernels with ceilings that
 * these measure on the device at hand.
 *  - Issue probes (kind RSAPRNG_PROBE_FMA_F64 .. RSAPRNG_PROBE_MUL_U32_U24):
 *    every lane of 8 waves per SIMD on every compute unit runs n loop trips of
 *    32 instructions of one class (8 independent dependency chains of 4), so
 *    the launch is bound by that class's issue rate.  The out pointers are
 *    ignored (a per-device sink of the library receives one word per lane).
 *    1 <= n <= 2^32.  *work = the lane-instructions of the class issued.
 *  - Store probes: n elements written to each of out_u64 and out_f64
 *    (device, 16-byte aligned, n a positive multiple of 2^20, n <= 2^36) with
 *    the chain-serial tile kernels' store patterns: one work-group per 2^20
 *    elements, 16-byte stores, each store instruction covering 1 KiB; 512
 *    lanes with c and r stores alternating (RSAPRNG_PROBE_STORE_TILE,
 *    non-temporal, as the kernels of two chunks of 8 indices per lane;
 *    RSAPRNG_PROBE_STORE_TILE_PLAIN, regular stores), or 256 lanes with a
 *    wave's eight c stores before its eight r stores
 *    (RSAPRNG_PROBE_STORE_BLOCK16, non-temporal, as the kernels of 16 indices
 *    per lane; RSAPRNG_PROBE_STORE_BLOCK16_PLAIN, regular stores); or a plain
 *    linear write (RSAPRNG_PROBE_STORE_LINEAR).  *work = the bytes written,
 *    16 n.
 * Enqueued on `stream`; the caller times the launch.  RSAPRNG_E_ARG for an
 * unknown kind or a bad n, RSAPRNG_E_ALIGN for misaligned store buffers.
 * ------------------------------------------------------------------------ */
#define RSAPRNG_PROBE_FMA_F64 0
#define RSAPRNG_PROBE_MUL_F64 1
#define RSAPRNG_PROBE_ADD_F64 2
#define RSAPRNG_PROBE_RNDNE_F64 3
#define RSAPRNG_PROBE_MAD_U64_U32 4
#define RSAPRNG_PROBE_MUL_LO_U32 5
#define RSAPRNG_PROBE_MUL_HI_U32 6
#define RSAPRNG_PROBE_ADD_U32 7
#define RSAPRNG_PROBE_CVT_F64_U32 8
#define RSAPRNG_PROBE_LSHL_ADD_U64 9
#define RSAPRNG_PROBE_MUL_U32_U24 10
#define RSAPRNG_PROBE_STORE_TILE 16
#define RSAPRNG_PROBE_STORE_LINEAR 17
#define RSAPRNG_PROBE_STORE_TILE_PLAIN 18
#define RSAPRNG_PROBE_STORE_BLOCK16 19
#define RSAPRNG_PROBE_STORE_BLOCK16_PLAIN 20
int rsaprng_probe(int kind, uint64_t n, uint64_t* out_u64, double* out_f64, double* work,
                  void* stream);

/* Library version string. */
const char* rsaprng_version(void);

#ifdef __cplusplus
}
#endif
#endif /* RSAPRNG_H */
