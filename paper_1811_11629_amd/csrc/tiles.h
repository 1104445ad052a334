// gfx950 kernels of the RSA-exponentiation generator.
//
// The work of a launch is a list of chains (the tiles of one request inside
// one 2^20 block) and T = WG * V * R consecutive indices per tile or step.
//
//   k_chain_setup  one wave per chain: the skip at the chain start,
//                  s0 a^S mod Q, by a product tree of the table a^(2^i) over
//                  the 64 lanes (eq. pseudoskip for the skips); for a block
//                  start also the block seed G_b = s0 a (a^{bB} - 1)/(a - 1),
//                  giving the message before the chain; fills tile -> chain.
//   k_sums         (two-pass) one wave per tile: the tile's skips
//                  (eq. congruentialgenerator1) summed mod n.
//   k_scan         (two-pass) one wave per chain: exclusive prefix of the tile
//                  sums, i.e. the message before every tile (m_k = m_{k-1} + s_k).
//   k_gen2/1/3     the tile kernels: V skips per lane, lane totals scanned
//                  across the wave with DPP moves, then per element
//                  c = m^e mod n (Montgomery-64 or CRT with binary64
//                  residues) and r = RN(c)/RN(n) with the 1.0 guard, stored to
//                  HBM through a per-wave LDS transpose (generate), folded into
//                  exact statistics flushed once per tile or chain (consume),
//                  or counted into the battery record (battery).  The message
//                  before a tile comes from k_scan (k_gen2), from a decoupled
//                  look-back over the chain's earlier tiles (k_gen1: atomic
//                  tile queue, tagged 64-bit words, relaxed agent-scope
//                  atomics, bounded wait), or from the carry of the previous
//                  step when one work-group walks the whole chain (k_gen3).
#pragma once
#include <type_traits>

#include "common.h"
#include "devmath.h"

namespace rsaprng {

__device__ __forceinline__ u64 wave_sum_mod(u64 v, u64 n) {
#pragma unroll
  for (int m = 1; m < 64; m <<= 1) v = addmod(v, __shfl_xor(v, m, 64), n);
  return v;
}

__device__ __forceinline__ u64 submod(u64 x, u64 y, u64 n) {
  return x >= y ? x - y : x + (n - y);
}

__device__ __forceinline__ u32 uniform(u32 v) { return __builtin_amdgcn_readfirstlane(v); }

// f(integral_constant<int, I>) for I = B .. E-1, each call its own instantiation.
template <int B, int E, class F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    static_for<B + 1, E>(f);
  }
}

// Read-only launch data (chains, instance records, per-tile and per-chunk
// prefixes) seen through the constant address space: with wave-uniform
// indices these become scalar loads, which do not wait on the wave's earlier
// vector stores the way vector loads do.
template <class T>
__device__ __forceinline__ const __attribute__((address_space(4))) T* cst(const T* p) {
  return (const __attribute__((address_space(4))) T*)p;
}

// Copy of a record through the constant address space, word by word.
template <class T>
__device__ __forceinline__ T load_cst(const T* p) {
  static_assert(sizeof(T) % 8 == 0, "record of 64-bit words");
  T out;
  const __attribute__((address_space(4))) u64* src = cst(reinterpret_cast<const u64*>(p));
  u64* dst = reinterpret_cast<u64*>(&out);
#pragma unroll
  for (int i = 0; i < (int)(sizeof(T) / 8); ++i) dst[i] = src[i];
  return out;
}

// 64-bit DPP move: lanes whose source is outside the row pattern (or whose row
// is masked off) receive 0.  With every row enabled the zero comes from the
// bound control (an out-of-range source reads 0), so no zeroed destination
// has to be prepared; masked-off rows keep the destination's old value, 0.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ u64 dpp64(u64 v) {
  u32 lo, hi;
  if constexpr (ROW_MASK == 0xf) {
    lo = (u32)__builtin_amdgcn_mov_dpp((int)lo32(v), CTRL, 0xf, 0xf, true);
    hi = (u32)__builtin_amdgcn_mov_dpp((int)hi32(v), CTRL, 0xf, 0xf, true);
  } else {
    lo = (u32)__builtin_amdgcn_update_dpp(0, (int)lo32(v), CTRL, ROW_MASK, 0xf, false);
    hi = (u32)__builtin_amdgcn_update_dpp(0, (int)hi32(v), CTRL, ROW_MASK, 0xf, false);
  }
  return ((u64)hi << 32) | lo;
}

// Inclusive scan mod n over the 64 lanes: row shifts by 1, 2, 4, 8 inside
// rows of 16, then the row-15 and row-31 broadcasts (full-rate VALU moves).
__device__ __forceinline__ u64 wave_scan_mod(u64 x, u64 n) {
  x = addmod(x, dpp64<0x111, 0xf>(x), n);  // row_shr:1
  x = addmod(x, dpp64<0x112, 0xf>(x), n);  // row_shr:2
  x = addmod(x, dpp64<0x114, 0xf>(x), n);  // row_shr:4
  x = addmod(x, dpp64<0x118, 0xf>(x), n);  // row_shr:8
  x = addmod(x, dpp64<0x142, 0xa>(x), n);  // row_bcast:15 into rows 1 and 3
  x = addmod(x, dpp64<0x143, 0xc>(x), n);  // row_bcast:31 into rows 2 and 3
  return x;
}

__device__ __forceinline__ u64 lane_value(u64 v, int lane) {
  const u32 lo = (u32)__builtin_amdgcn_readlane((int)lo32(v), lane);
  const u32 hi = (u32)__builtin_amdgcn_readlane((int)hi32(v), lane);
  return ((u64)hi << 32) | lo;
}

__device__ __forceinline__ double lane_value_f64(double v, int lane) {
  return __longlong_as_double((long long)lane_value((u64)__double_as_longlong(v), lane));
}

// ---------------------------------------------------------------------------
// look-back words: (tag << 32) | half, two words per 64-bit value
// ---------------------------------------------------------------------------
__device__ __forceinline__ void publish(u64* w, u32 tag, u64 v) {
  u64 a = ((u64)tag << 32) | lo32(v);
  u64 b = ((u64)tag << 32) | hi32(v);
  __hip_atomic_store(w, a, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __hip_atomic_store(w + 1, b, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ bool try_read(const u64* w, u32 tag, u64& v) {
  u64 a = __hip_atomic_load(const_cast<u64*>(w), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  u64 b = __hip_atomic_load(const_cast<u64*>(w + 1), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (hi32(a) != tag || hi32(b) != tag) return false;
  v = ((u64)lo32(b) << 32) | lo32(a);
  return true;
}

// Exclusive prefix (mod n) of tile t: the inclusive value of the nearest
// predecessor that has one plus the aggregates in between.  One full wave;
// the chain's first tile always publishes an inclusive value.
__device__ u64 look_back(const LaunchArgs& a, u32 t, u32 first, u32 tag, u64 n, int lane) {
  u64 acc = 0;
  long pos = (long)t - 1;
  u32 spins = 0;
  for (;;) {
    long u = pos - lane;
    bool valid = u >= (long)first;
    bool hasI = false, hasA = false;
    u64 vi = 0, va = 0;
    for (;;) {
      if (valid && !hasI) {
        hasI = try_read(a.lb + 4 * u + 2, tag, vi);
        if (!hasI && !hasA) hasA = try_read(a.lb + 4 * u, tag, va);
      }
      bool ready = !valid || hasI || hasA;
      if (__all(ready)) break;
      if (++spins > a.spin_limit) {
        if (lane == 0) atomicOr(&a.ctl->err, 1u);
        return acc;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    u64 imask = __ballot(valid && hasI);
    int stop = imask ? __ffsll((unsigned long long)imask) - 1 : 64;
    u64 contrib = 0;
    if (valid) contrib = lane < stop ? va : (lane == stop ? vi : 0);
    acc = addmod(acc, lane_value(wave_scan_mod(contrib, n), 63), n);
    if (imask) return acc;
    pos -= 64;
  }
}

// ---------------------------------------------------------------------------
// encryption of one message
// ---------------------------------------------------------------------------
// The instance's reductions mod p and mod q (devmath.h, fold_split and residue).
__device__ __forceinline__ double fold_p(double H, const rsaprng_params& P) {
  return fold_split(H, P.pd, P.kp_lo, P.kp_hi, P.kp_quo);
}
__device__ __forceinline__ double fold_q(double H, const rsaprng_params& P) {
  return fold_split(H, P.qd, P.kq_lo, P.kq_hi, P.kq_quo);
}
__device__ __forceinline__ double res_p(u64 m, const rsaprng_params& P) {
  return residue(m, P.pd, P.pinv, P.kp_lo, P.kp_hi, P.kp_quo);
}
__device__ __forceinline__ double res_q(u64 m, const rsaprng_params& P) {
  return residue(m, P.qd, P.qinv, P.kq_lo, P.kq_hi, P.kq_quo);
}
__device__ __forceinline__ double ratio_of(double cd, const rsaprng_params& P) {
  return ratio(cd, P.nd, P.nrcp, P.nrcp_lo);
}

// CRT form from the residues of m: m^E mod p and mod q, then Garner.  For
// E >= 2 the residues may be unreduced (|x| < 2^42: the ladder opens with a
// squaring), otherwise they must lie in (-P, P).
template <u32 E>
__device__ __forceinline__ u64 encrypt_res(double mp, double mq, const rsaprng_params& P,
                                           double& cd) {
  double cp, cq;
  if constexpr (E != 0) {
    cp = fp_pow<E>(mp, P.pd, P.pinv);
    cq = fp_pow<E>(mq, P.qd, P.qinv);
  } else {
    // generic ladders with the exponents of each prime (equal to e unless the
    // instance has different exponents mod p and mod q)
    cp = fp_pow_rt(mp, P.pd, P.pinv, P.ep);
    cq = fp_pow_rt(mq, P.qd, P.qinv, P.eq);
  }
  return garner(cp, cq, P.pd, P.qd, P.pinv, P.qinv, P.gp_lo, P.gp_hi, P.gp_quo, P.q, cd);
}

template <int VAR, u32 E>
__device__ __forceinline__ u64 encrypt(u64 m, const rsaprng_params& P, double& cd) {
  if constexpr (VAR == kVariantMont) {
    u64 c;
    if constexpr (E != 0)
      c = mont_encrypt<E>(m, P.n, P.ninv, P.ce);
    else
      c = mont_encrypt_rt(m, P.n, P.ninv, P.ce, P.e);
    cd = u64_to_f64_rn(c);
    return c;
  } else {
    double mp, mq;
    if constexpr (E >= 2) {  // the ladder starts with a squaring
      mp = residue_lazy(m, P.pd, P.kp_lo, P.kp_hi, P.kp_quo);
      mq = residue_lazy(m, P.qd, P.kq_lo, P.kq_hi, P.kq_quo);
    } else {
      mp = res_p(m, P);
      mq = res_q(m, P);
    }
    return encrypt_res<E>(mp, mq, P, cd);
  }
}

// Adds r 2^128 (r = 0 or 2^-64 <= r < 1, so r 2^128 = mant 2^(ex - 947) is an
// integer with the shift in [12, 75]) to the 128-bit sum lo + 2^64 hi, counting
// the carries out of hi in hc.  For r >= 2^-12 (all but about one output in
// 4096) the low word is zero and r 2^64 = mant 2^(ex - 1011) < 2^64 is added to
// hi alone; the rest take the full shift.
__device__ __forceinline__ void add_fixed128(double r, u64& lo, u64& hi, u32& hc) {
  const u64 bits = (u64)__double_as_longlong(r);
  const u32 ex = (u32)(bits >> 52);
  const u64 mant = (bits & 0xfffffffffffffull) | (1ull << 52);
  if (ex >= 1011) {
    const u64 v = mant << (ex - 1011);
    const u64 t = hi + v;
    hc += t < v;
    hi = t;
  } else if (ex != 0) {
    const u32 sh = ex - 947;                  // in [12, 64)
    const u64 vl = mant << sh;
    const u64 vh = mant >> (64 - sh);         // < 2^53
    const u64 t = lo + vl;
    const u64 h2 = vh + (t < vl);             // < 2^53 + 1: no wrap
    lo = t;
    const u64 t2 = hi + h2;
    hc += t2 < h2;
    hi = t2;
  }
}

// ---------------------------------------------------------------------------
// Message sources of one lane's V consecutive indices.  enc<VAR, E>(i, ...)
// encrypts the i-th message; callers take i = 0, 1, ..., V-1 in order.
// ---------------------------------------------------------------------------
// Exact messages: m_i = (pre + X_i) mod n, X_i the running skip sums mod n.
template <int V>
struct MsgExact {
  u64 pre, n;
  const u64 (&X)[V];
  template <int VAR, u32 E>
  __device__ __forceinline__ u64 enc(int i, const rsaprng_params& P, double& cd) {
    return encrypt<VAR, E>(addmod(pre, X[i], n), P, cd);
  }
};

// x (an integer-valued double, |x| < 2^52) reduced into (-P, P).
__device__ __forceinline__ double reduce_res(double x, double P, double Pinv) {
  return __fma_rn(-__builtin_rint(x * Pinv), P, x);
}

// Residue messages (CRT variant).  With the lane's skips s_0..s_{V-1} and the
// residues bp, bq of the message before its first index (in (-p, p), (-q, q)),
// m_i is congruent to b + s_0 + ... + s_i.  Only m mod p and m mod q enter the
// encryption, so no 64-bit modular addition is done: each skip s = h 2^32 + l
// adds fold_p(h) + l to the running residue mp (fold_p(h) in (-p, p)), so after
// V <= 16 skips |mp| < p + 16 (p + 2^32) < 2^38, a valid input of the ladder's
// opening squaring (below 2^42), and of reduce_res otherwise (likewise mod q).
template <int V>
struct MsgRes {
  const u64 (&S)[V];
  double Ap, Aq;  // bp, bq on entry; then the residues of the latest message
  template <int VAR, u32 E>
  __device__ __forceinline__ u64 enc(int i, const rsaprng_params& P, double& cd) {
    static_assert(V <= 16, "residue bound");
    const double h = (double)hi32(S[i]);
    const double l = (double)lo32(S[i]);
    Ap += fold_p(h, P) + l;
    Aq += fold_q(h, P) + l;
    double mp = Ap;
    double mq = Aq;
    if constexpr (E < 2) {  // no opening squaring: Garner needs reduced residues
      mp = reduce_res(mp, P.pd, P.pinv);
      mq = reduce_res(mq, P.qd, P.qinv);
    }
    return encrypt_res<E>(mp, mq, P, cd);
  }
};

// The same, walking the lane's skips from its first one as the indices are
// taken (nothing kept from an earlier walk).
template <int V>
struct MsgResWalk {
  u64 s;
  double Ap, Aq;  // bp, bq on entry; then the residues of the latest message
  template <int VAR, u32 E>
  __device__ __forceinline__ u64 enc(int i, const rsaprng_params& P, double& cd) {
    static_assert(V <= 16, "residue bound");
    if (i) s = lcg_next(s);
    const double h = (double)hi32(s);
    const double l = (double)lo32(s);
    Ap += fold_p(h, P) + l;
    Aq += fold_q(h, P) + l;
    double mp = Ap;
    double mq = Aq;
    if constexpr (E < 2) {
      mp = reduce_res(mp, P.pd, P.pinv);
      mq = reduce_res(mq, P.qd, P.qinv);
    }
    return encrypt_res<E>(mp, mq, P, cd);
  }
};

// Exact messages, walking: m_i = (pre + s_0 + ... + s_i) mod n.
template <int V>
struct MsgExactWalk {
  u64 pre, n, s;
  u64 x = 0;
  template <int VAR, u32 E>
  __device__ __forceinline__ u64 enc(int i, const rsaprng_params& P, double& cd) {
    if (i) s = lcg_next(s);
    x = addmod(x, skip_mod_n(s, n), n);
    return encrypt<VAR, E>(addmod(pre, x, n), P, cd);
  }
};

// Two 64-bit words as one 16-byte vector (non-temporal stores of pairs).
typedef u64 u64x2 __attribute__((ext_vector_type(2)));

// Row stride (64-bit words) of a wave's transpose buffer: 8 values per lane
// plus one word of padding against LDS bank conflicts.
constexpr int kXRow = 9;

// Stores a wave's 64 x 8 transposed block x (row = lane, 8 consecutive outputs)
// to dst[0 .. 512).  With dst 16-byte aligned, store j writes elements 128 j +
// 2 lane and the next (rows 16 j + lane / 4, columns 2 (lane % 4) and the
// next): each 16-byte store instruction covers 1 KiB of contiguous output, with
// the non-temporal hint (the outputs are not read again by the kernel).
// Otherwise (an output range packed at an odd element) store j writes element
// 64 j + lane: each 8-byte store instruction covers 512 contiguous bytes.
// A16: 1 or 0 when the caller knows the alignment, -1 to test it here (a
// wave-uniform branch).
// src: (lane / 4) kXRow + 2 (lane % 4), formed by the caller before its wave
// barrier.
template <int A16>
__device__ __forceinline__ void store_chunk(u64* dst, const u64* x, int src, int lane) {
  if (A16 == 1 || (A16 == -1 && ((uintptr_t)dst & 15) == 0)) {
#pragma unroll
    for (int j = 0; j < 4; ++j)
      __builtin_nontemporal_store(u64x2{x[j * 16 * kXRow + src], x[j * 16 * kXRow + src + 1]},
                                  reinterpret_cast<u64x2*>(dst + (u64)j * 128 + 2 * lane));
  } else {
    const int src8 = (lane >> 3) * kXRow + (lane & 7);
#pragma unroll
    for (int j = 0; j < 8; ++j) dst[(u64)j * 64 + lane] = x[j * 8 * kXRow + src8];
  }
}

// Row stride of the 64 x 16 block of a lane holding 16 consecutive indices: 16
// values plus one word of padding.  The block fits in the wave's share of the
// transpose buffer (2 x 64 x kXRow words), and c and then r pass through it.
constexpr int kXRow16 = 17;
static_assert(64 * kXRow16 <= 2 * 64 * kXRow, "one 64 x 16 block per wave");

// Stores a wave's 64 x 16 transposed block x (row = lane, 16 consecutive
// outputs) to dst[0 .. 1024).  With dst 16-byte aligned, store j writes
// elements 128 j + 2 lane and the next (row 8 j + lane / 8, columns 2 (lane %
// 8) and the next): 1 KiB of contiguous output per store instruction, as for
// the 64 x 8 blocks.  Otherwise store j writes element 64 j + lane (row 4 j +
// lane / 16, column lane % 16), 512 contiguous bytes per instruction.  A16 as
// for store_chunk.
template <int A16>
__device__ __forceinline__ void store_chunk16(u64* dst, const u64* x, int lane) {
  if (A16 == 1 || (A16 == -1 && ((uintptr_t)dst & 15) == 0)) {
    const int src = (lane >> 3) * kXRow16 + 2 * (lane & 7);
#pragma unroll
    for (int j = 0; j < 8; ++j)
      __builtin_nontemporal_store(
          u64x2{x[j * 8 * kXRow16 + src], x[j * 8 * kXRow16 + src + 1]},
          reinterpret_cast<u64x2*>(dst + (u64)j * 128 + 2 * lane));
  } else {
    const int src8 = (lane >> 4) * kXRow16 + (lane & 15);
#pragma unroll
    for (int j = 0; j < 16; ++j) dst[(u64)j * 64 + lane] = x[j * 4 * kXRow16 + src8];
  }
}

__device__ __forceinline__ void wave_sync_lds() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ---------------------------------------------------------------------------
// Statistical battery (fused consumer), chain-serial kernel only.  Tuples live
// inside aligned blocks of 8 indices, maxima in aligned blocks of 32, gap runs
// in aligned blocks of 64 and collision trials in aligned blocks of 2^14 (a
// block counts when all its indices are requested), so the counts do not
// depend on the tiling.  Large tables (frequency, serial) take device-scope
// atomics; the small ones (poker, maxima, runs) and the trial's urn bitmap
// live in the work-group's LDS and are flushed per chain or per trial.
// ---------------------------------------------------------------------------
constexpr int kBatPoker = 0;                 // LDS counts: poker classes [0, 8)
constexpr int kBatMax = 8;                   // maxima bins [8, 1032)
constexpr int kBatRuns = kBatMax + 1024;     // runs[b][L - 1] [1032, 1160)
constexpr int kBatLds = kBatRuns + 128;
constexpr int kTrialLog2 = 14;               // 2^14 balls per collision trial
constexpr int kUrnWords = (1 << 20) / 32;    // 2^20 urns as a bitmap
// leading bits of a step (at most 8192 indices), behind the previous step's
// last 32, and one word of slack for the funnel shift's upper operand
constexpr int kMsbWords = 8192 / 32 + 2;

__device__ __forceinline__ u32 bin_of(double r, double b, u32 nb) {
  const u32 x = (u32)(r * b);
  return x < nb ? x : nb - 1;
}

__device__ __forceinline__ void bat_add(u32* p) {
  __hip_atomic_fetch_add(p, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <int WG, int MODE>
struct TileShared;

// Counts of one lane's 8 consecutive values r[0..8), standing at absolute
// indices laneStart .. laneStart + 7, of which [k0, last] are requested; the 64
// lanes of the wave hold 512 consecutive indices (a chunk, aligned to 512).
template <int WG>
__device__ __forceinline__ void battery_count(const LaunchArgs& a, TileShared<WG, kModeBattery>& sh,
                                              u64 k0, u64 last, const double (&r)[8],
                                              u64 laneStart) {
  rsaprng_battery* const B = a.battery;
  const int lane = threadIdx.x & 63;
  // the chunk lies inside one collision trial
  const u64 kt = laneStart >> kTrialLog2 << kTrialLog2;
  const bool trial = kt >= k0 && kt <= last && last - kt >= (1ull << kTrialLog2) - 1;
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const u64 k = laneStart + i;
    const u32 u = bin_of(r[i], 1048576.0, 1u << 20);
    if (k >= k0 && k <= last) bat_add(&B->freq[u]);
    if (trial)
      __hip_atomic_fetch_or(&sh.urn[u >> 5], 1u << (u & 31), __ATOMIC_RELAXED,
                            __HIP_MEMORY_SCOPE_WORKGROUP);
  }
  const bool full = laneStart >= k0 && laneStart <= last && last - laneStart >= 7;
  double mx = 0.0;
#pragma unroll
  for (int i = 0; i < 8; ++i) mx = r[i] > mx ? r[i] : mx;
  // poker: the five classes counted per wave (one LDS add per class)
  u32 hand = 0;
#pragma unroll
  for (int j = 0; j < 5; ++j) hand |= 1u << bin_of(r[j], 16.0, 16);
  const u32 distinct = __builtin_popcount(hand);
#pragma unroll
  for (u32 d = 1; d <= 5; ++d) {
    const u64 m = __ballot(full && distinct == d);
    if (lane == 0 && m) atomicAdd(&sh.bh[kBatPoker + d], (u32)__popcll(m));
  }
  if (full) {
#pragma unroll
    for (int t = 0; t < 4; ++t)
      bat_add(&B->serial2[bin_of(r[2 * t], 1024.0, 1024) * 1024 + bin_of(r[2 * t + 1], 1024.0, 1024)]);
#pragma unroll
    for (int t = 0; t < 2; ++t)
      bat_add(&B->serial3[(bin_of(r[3 * t], 100.0, 100) * 100 + bin_of(r[3 * t + 1], 100.0, 100)) * 100 +
                          bin_of(r[3 * t + 2], 100.0, 100)]);
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      u32 c = 0;
#pragma unroll
      for (int j = 0; j < 4; ++j) c = c * 32 + bin_of(r[4 * t + j], 32.0, 32);
      bat_add(&B->serial4[c]);
    }
    u32 c5 = 0, c6 = 0;
#pragma unroll
    for (int j = 0; j < 5; ++j) c5 = c5 * 16 + bin_of(r[j], 16.0, 16);
#pragma unroll
    for (int j = 0; j < 6; ++j) c6 = c6 * 10 + bin_of(r[j], 10.0, 10);
    bat_add(&B->serial5[c5]);
    bat_add(&B->serial6[c6]);
  }
  // maximum of 32: the four lanes holding one aligned block of 32 indices
  bool all = full;
#pragma unroll
  for (int m = 1; m < 4; m <<= 1) {
    const double o = __shfl_xor(mx, m, 64);
    mx = o > mx ? o : mx;
    all = (__shfl_xor((int)all, m, 64) != 0) && all;
  }
  if (all && (lane & 3) == 0) {
    double x = mx;
#pragma unroll
    for (int j = 0; j < 5; ++j) x = x * x;  // M^32
    atomicAdd(&sh.bh[kBatMax + bin_of(x, 1024.0, 1024)], 1u);
  }
  // gaps: the run of b = [r > 1/2] that starts at an aligned block of 64
  // (lanes g0 .. g0 + 7): full lanes continue it, the first other lane ends it
  u32 bits = 0;
#pragma unroll
  for (int i = 0; i < 8; ++i) bits |= (r[i] > 0.5 ? 1u : 0u) << i;
  const int g0 = lane & ~7;
  const u32 b0 = (u32)__shfl((int)(bits & 1u), g0, 64);
  const u32 same = b0 ? bits : (~bits & 0xffu);  // 1 where the bit equals b0
  const u32 t = same == 0xffu ? 8u : (u32)__builtin_ctz(~same);
  const u32 fullm = (u32)(__ballot(t == 8u) >> g0) & 0xffu;
  const u32 m = fullm == 0xffu ? 8u : (u32)__builtin_ctz(~fullm);
  const u32 tm = (u32)__shfl((int)t, g0 + (m < 8u ? (int)m : 7), 64);
  const u64 k64 = laneStart - (u64)(lane & 7) * 8;
  const bool blk64 = k64 >= k0 && k64 <= last && last - k64 >= 63;
  if ((lane & 7) == 0 && blk64) atomicAdd(&sh.bh[kBatRuns + b0 * 64 + (m < 8u ? 8u * m + tm : 64u) - 1], 1u);
  // the leading bits floor(2 r) of the lane's 8 values: one byte of the step's
  // bit string (steps of 2^tile_log2 indices, aligned to their size)
  u32 lead = 0;
#pragma unroll
  for (int i = 0; i < 8; ++i) lead |= (r[i] >= 0.5 ? 1u : 0u) << i;
  const u32 off8 = (u32)((laneStart & ((1ull << a.tile_log2) - 1)) >> 3);
  reinterpret_cast<unsigned char*>(sh.msb + 1)[off8] = (unsigned char)lead;
}

// Leading-bit collision trials (rsaprng.h): after a step [base, base + T)
// whose bytes are in sh.msb[1 ..], behind the previous step's last 32 bits in
// sh.msb[0], every ball whose last index lies in the step.  A trial counts
// when all its indices lie in [k0, last]; its bitmap (work-group slot `slot`
// of a.urn2, by trial parity) is cleared at the step of its first ball, and
// its distinct urns are read out at the step of its last.  Called by every
// thread of the work-group, after every byte of the step is written; the next
// step's bytes may be written as soon as it returns (only sh.msb[0] is written
// after its last barrier).
template <int WG>
__device__ void msb_step(const LaunchArgs& a, TileShared<WG, kModeBattery>& sh, u64 base, u32 T,
                         u64 k0, u64 last, u32 slot) {
  const u64 blk = base & ~(kBlock - 1);
  const u64 rel = base - blk;                     // a multiple of T
  const u64 g_lo = rel / kMsbBall;                // first ball ending at or after base
  u64 g_hi = (rel + T) / kMsbBall;                // first ball ending after the step
  constexpr u64 kBalls = (u64)kMsbTrials << kTrialLog2;
  if (g_hi > kBalls) g_hi = kBalls;
  u32* const bm = a.urn2 + (u64)slot * kUrn2Words;
  const auto counted = [&](u64 j) {
    const u64 ts = blk + j * kMsbTrial;
    return ts >= k0 && ts <= last && last - ts >= kMsbTrial - 1;
  };
#pragma unroll
  for (int j = 0; j < kMsbTrials; ++j) {
    const u64 g0 = (u64)j << kTrialLog2;
    if (g0 >= g_lo && g0 < g_hi && counted(j)) {
      u32* b = bm + (j & 1) * kUrnWords;
      for (int i = threadIdx.x; i < kUrnWords; i += WG) b[i] = 0;
      if (threadIdx.x == 0) sh.dist2[j & 1] = 0;
    }
  }
  __syncthreads();  // the step's bytes, the cleared bitmaps
  // the step's last 32 bits, kept for the next step's first balls (written to
  // sh.msb[0] once every ball below has read it; the next step's bytes may
  // already be arriving then, so it is read now)
  const u32 tail = threadIdx.x == 0 ? sh.msb[T / 32] : 0u;
  for (u64 g = g_lo + threadIdx.x; g < g_hi; g += WG) {
    const u64 j = g >> kTrialLog2;
    if (!counted(j)) continue;
    const u32 o = (u32)(g * kMsbBall + 32 - rel);  // ball's first bit, counted from base - 32
    const u32 w = o >> 5;
    const u32 urn = __builtin_amdgcn_alignbit(sh.msb[w + 1], sh.msb[w], o & 31) & 0xfffffu;
    const u32 bit = 1u << (urn & 31);
    const u32 old = __hip_atomic_fetch_or(bm + (j & 1) * kUrnWords + (urn >> 5), bit,
                                          __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (!(old & bit)) atomicAdd(&sh.dist2[j & 1], 1u);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int j = 0; j < kMsbTrials; ++j) {
      const u64 gl = (((u64)j + 1) << kTrialLog2) - 1;
      if (gl >= g_lo && gl < g_hi && counted(j)) {
        const u32 c = (1u << kTrialLog2) - sh.dist2[j & 1];
        bat_add(&a.battery->coll_msb[c < 255 ? c : 255]);
      }
    }
    sh.msb[0] = tail;
  }
}

template <int WG, int V, int VAR, u32 E, class Msg>
__device__ __forceinline__ void battery_outputs(const LaunchArgs& a,
                                                TileShared<WG, kModeBattery>& sh, const Chain& C,
                                                const rsaprng_params& P, Msg msg, u64 laneStart) {
  static_assert(V == 8, "a lane holds one block of 8; 8 lanes hold a block of 64");
  double rv[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    double cd;
    (void)msg.template enc<VAR, E>(i, P, cd);
    rv[i] = ratio_of(cd, P);
  }
  battery_count<WG>(a, sh, C.k0, C.last, rv, laneStart);
}

template <int WG, int MODE>
struct TileShared {
  u32 tile;
  u64 pre;
  u64 wave_tot[WG / 64];
  u64 red[MODE == kModeConsume ? (WG / 64) * 7 : 1];
  u32 hist[MODE == kModeConsume ? 1024 : 1];
  // consume: per-thread running sums (the 32-bit digit sums d0..d4 of the
  // fixed-point sum, r < 0.5, count), acc[j WG + thread], flushed to the
  // record by consume_flush
  u64 acc[MODE == kModeConsume ? 7 * WG : 1];
  // generate: per wave, two 64 x 8 blocks (c, then r) for the coalescing transpose
  u64 xbuf[MODE == kModeGenerate ? 2 * (WG / 64) * 64 * kXRow : 1];
  // battery: the current collision trial's urns, and the small tables
  u32 urn[MODE == kModeBattery ? kUrnWords : 1];
  u32 bh[MODE == kModeBattery ? kBatLds : 1];
  // battery: the step's leading bits and the distinct urns of the two
  // leading-bit trials in flight (by parity)
  u32 msb[MODE == kModeBattery ? kMsbWords : 1];
  u32 dist2[2];
};

// Encryption and output of one tile for exponent E (0 = any exponent).  FAST:
// every index of the tile is requested and both outputs are 16-byte aligned at
// every lane's first index, so pairs are stored without predicates.
template <int WG, int V, int VAR, int MODE, u32 E, bool FAST, int A16 = -1, bool XB16 = false,
          class Msg>
__device__ __forceinline__ void tile_outputs(const LaunchArgs& a, TileShared<WG, MODE>& sh,
                                             const Chain& C, const rsaprng_params& P, Msg msg,
                                             u64 laneStart) {
  const bool full = FAST || (laneStart >= C.k0 && laneStart + (V - 1) <= C.last);
  if constexpr (MODE == kModeGenerate) {
    u64* const oc = a.out_c;
    double* const orr = a.out_r;
    if constexpr (FAST && V == 8) {
      // Each lane's 8 results go to its row of the wave's LDS buffers (c and r)
      // as they are produced, then store_chunk writes them coalesced.  No
      // result waits in registers.
      const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
      u64* xc = sh.xbuf + wave * (2 * 64 * kXRow);
      u64* xr = xc + 64 * kXRow;
#pragma unroll
      for (int i = 0; i < V; ++i) {
        double cd;
        const u64 c = msg.template enc<VAR, E>(i, P, cd);
        xc[lane * kXRow + i] = c;
        xr[lane * kXRow + i] = (u64)__double_as_longlong(ratio_of(cd, P));
      }
      const u64 chunk0 = C.out_off + (laneStart - (u64)lane * V - C.k0);
      const int src = (lane >> 2) * kXRow + 2 * (lane & 3);
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      if (oc) store_chunk<A16>(oc + chunk0, xc, src, lane);
      if (orr) store_chunk<A16>(reinterpret_cast<u64*>(orr) + chunk0, xr, src, lane);
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    } else if constexpr (FAST && V == 16 && XB16) {
      // (the kernels specialised to one exponent) The lane's 16 ciphertexts
      // go to its row of the wave's 64 x 16 block and are stored from there;
      // its 16 ratios wait in registers meanwhile and then take the same
      // block.
      const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
      u64* x = sh.xbuf + wave * (2 * 64 * kXRow);
      u64 rv[V];
#pragma unroll
      for (int i = 0; i < V; ++i) {
        double cd;
        x[lane * kXRow16 + i] = msg.template enc<VAR, E>(i, P, cd);
        rv[i] = (u64)__double_as_longlong(ratio_of(cd, P));
      }
      const u64 chunk0 = C.out_off + (laneStart - (u64)lane * V - C.k0);
      wave_sync_lds();
      if (oc) store_chunk16<A16>(oc + chunk0, x, lane);
      if (orr) {
        wave_sync_lds();
#pragma unroll
        for (int i = 0; i < V; ++i) x[lane * kXRow16 + i] = rv[i];
        wave_sync_lds();
        store_chunk16<A16>(reinterpret_cast<u64*>(orr) + chunk0, x, lane);
      }
      wave_sync_lds();
    } else if constexpr (FAST) {
      const u64 off0 = C.out_off + (laneStart - C.k0);
#pragma unroll
      for (int i = 0; i < V; i += 2) {
        double cd0, cd1;
        const u64 c0 = msg.template enc<VAR, E>(i, P, cd0);
        const u64 c1 = msg.template enc<VAR, E>(i + 1, P, cd1);
        if (oc) *reinterpret_cast<ulonglong2*>(oc + off0 + i) = make_ulonglong2(c0, c1);
        if (orr)
          *reinterpret_cast<double2*>(orr + off0 + i) =
              make_double2(ratio_of(cd0, P), ratio_of(cd1, P));
      }
    } else {
#pragma unroll
      for (int i = 0; i < V; ++i) {
        const u64 k = laneStart + i;
        double cd;
        const u64 c = msg.template enc<VAR, E>(i, P, cd);
        if (k >= C.k0 && k <= C.last) {
          const u64 off = C.out_off + (k - C.k0);
          if (oc) oc[off] = c;
          if (orr) orr[off] = ratio_of(cd, P);
        }
      }
    }
  } else if constexpr (MODE == kModeBattery) {
    battery_outputs<WG, V, VAR, E>(a, sh, C, P, msg, laneStart);
  } else {
    // the lane's exact sum of r 2^128 over its V indices as lo + 2^64 hi +
    // 2^128 hc, then added to the thread's running digit sums
    u64 lo = 0, hi = 0;
    u32 hc = 0, lt = 0, cnt = 0;
#pragma unroll
    for (int i = 0; i < V; ++i) {
      const u64 k = laneStart + i;
      double cd;
      (void)msg.template enc<VAR, E>(i, P, cd);
      const double r = ratio_of(cd, P);
      if (full || (k >= C.k0 && k <= C.last)) {
        add_fixed128(r, lo, hi, hc);
        lt += r < 0.5;
        if (!full) cnt += 1;
        atomicAdd(&sh.hist[(int)(r * 1024.0)], 1u);
      }
    }
    if (full) cnt = V;
    u64* const acc = sh.acc + threadIdx.x;
    acc[0] += lo32(lo);
    acc[WG] += hi32(lo);
    acc[2 * WG] += lo32(hi);
    acc[3 * WG] += hi32(hi);
    acc[4 * WG] += hc;
    acc[5 * WG] += lt;
    acc[6 * WG] += cnt;
  }
}

// Consume: the work-group's running sums and histogram added to stats record
// `slot` and cleared.  Called by every thread of the work-group, after the
// last chunk of a tile (or chain) that reduced into this record.  Per thread
// each digit sum stays below 2^32 times the thread's outputs (at most 2^14 per
// chain of 2^20), so every total below is far from 2^64.
template <int WG>
__device__ __forceinline__ void consume_flush(const LaunchArgs& a, TileShared<WG, kModeConsume>& sh,
                                              u32 slot) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  u64 v[7];
#pragma unroll
  for (int j = 0; j < 7; ++j) {
    v[j] = sh.acc[j * WG + threadIdx.x];
    sh.acc[j * WG + threadIdx.x] = 0;
  }
#pragma unroll
  for (int m = 1; m < 64; m <<= 1) {
#pragma unroll
    for (int j = 0; j < 7; ++j) v[j] += __shfl_xor(v[j], m, 64);
  }
  if (lane == 0) {
#pragma unroll
    for (int j = 0; j < 7; ++j) sh.red[wave * 7 + j] = v[j];
  }
  __syncthreads();
  rsaprng_stats* st = a.stats + slot;
  if (threadIdx.x == 0) {
    u64 s[5] = {0, 0, 0, 0, 0}, tl = 0, tc = 0;
    for (int w = 0; w < WG / 64; ++w) {
      for (int j = 0; j < 5; ++j) s[j] += sh.red[w * 7 + j];
      tl += sh.red[w * 7 + 5];
      tc += sh.red[w * 7 + 6];
    }
    // carry-normalise into 32-bit digits so each atomic adds < 2^32
    u64 carry = 0;
    u32 dig[6];
    for (int j = 0; j < 5; ++j) {
      u64 v = s[j] + carry;
      dig[j] = lo32(v);
      carry = v >> 32;
    }
    dig[5] = lo32(carry);
    for (int j = 0; j < 6; ++j)
      if (dig[j]) atomicAdd((unsigned long long*)&st->acc32[j], (unsigned long long)dig[j]);
    if (tl) atomicAdd((unsigned long long*)&st->lt_half, (unsigned long long)tl);
    if (tc) atomicAdd((unsigned long long*)&st->count, (unsigned long long)tc);
  }
  for (int b = threadIdx.x; b < 1024; b += WG) {
    const u32 h = sh.hist[b];
    if (h) {
      atomicAdd((unsigned long long*)&st->hist[b], (unsigned long long)h);
      sh.hist[b] = 0;
    }
  }
  // No wave may add to the histogram or the sums of the next tile (possibly
  // another record's) before every bin of this one is flushed.
  __syncthreads();
}

// Battery: the collision trial that just ended (all of its 2^14 indices
// requested): C = 2^14 - (urns hit), then the bitmap is cleared.  Called by
// every thread of the work-group.
template <int WG>
__device__ __forceinline__ void trial_flush(const LaunchArgs& a, TileShared<WG, kModeBattery>& sh) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  u32 hit = 0;
  for (int i = threadIdx.x; i < kUrnWords; i += WG) {
    hit += __builtin_popcount(sh.urn[i]);
    sh.urn[i] = 0;
  }
#pragma unroll
  for (int m = 1; m < 64; m <<= 1) hit += __shfl_xor(hit, m, 64);
  if (lane == 0) sh.wave_tot[wave] = hit;
  __syncthreads();
  if (threadIdx.x == 0) {
    u64 distinct = 0;
    for (int w = 0; w < WG / 64; ++w) distinct += sh.wave_tot[w];
    const u64 c = (1ull << kTrialLog2) - distinct;
    bat_add(&a.battery->coll[c < 255 ? c : 255]);
  }
  __syncthreads();
}

// Battery: the work-group's small tables added to the record and cleared.
template <int WG>
__device__ __forceinline__ void battery_flush(const LaunchArgs& a, TileShared<WG, kModeBattery>& sh) {
  __syncthreads();
  rsaprng_battery* const B = a.battery;
  for (int i = threadIdx.x; i < kBatLds; i += WG) {
    const u32 v = sh.bh[i];
    if (v) {
      u32* dst = i < kBatMax ? &B->poker[i - kBatPoker]
                             : (i < kBatRuns ? &B->maxt[i - kBatMax] : &B->runs[0][0] + (i - kBatRuns));
      __hip_atomic_fetch_add(dst, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      sh.bh[i] = 0;
    }
  }
  __syncthreads();
}

// Walk of one lane: V skips from s_first (eq. congruentialgenerator1), running
// sums mod n in X.  Returns the lane total.
template <int V>
__device__ __forceinline__ u64 walk(u64 s_first, u64 n, u64 (&X)[V]) {
  u64 s = s_first;
  u64 x = 0;
#pragma unroll
  for (int i = 0; i < V; ++i) {
    if (i) s = lcg_next(s);
    x = addmod(x, skip_mod_n(s, n), n);
    X[i] = x;
  }
  return x;
}

// The lane total of V skips as H 2^32 + L, the skips kept in S[0..V) when
// KEEP.  Two skips (each below 2^63) add without overflow; the pair sums go
// into a 64-bit accumulator with a carry count, so the total S = carry 2^64 +
// acc (below V 2^63) gives H = carry 2^32 + hi32(acc) < 2^35 and L = lo32(acc)
// exactly.  (A lazy walk whose values may exceed 2^63 is redone, so the bound
// holds for every accepted walk.)
template <int V, bool KEEP, bool LAZY>
__device__ __forceinline__ void walk_sum_run(u64 s_first, u64* S, double& H, double& L,
                                             u32& top) {
  static_assert(V % 2 == 0 && V <= 16, "pairs of skips; H below 2^35");
  u64 s = s_first;
  u64 acc = 0;
  u32 carry = 0;
#pragma unroll
  for (int i = 0; i < V; i += 2) {
    if (i) s = walk_step<LAZY>(s, top);
    const u64 s1 = walk_step<LAZY>(s, top);
    if constexpr (KEEP) {
      S[i] = s;
      S[i + 1] = s1;
    }
    const u64 pair = s + s1;
    const u64 t = acc + pair;
    carry += t < pair;
    acc = t;
    s = s1;
  }
  H = __fma_rn((double)carry, 4294967296.0, (double)hi32(acc));
  L = (double)lo32(acc);
}

template <int V, bool KEEP>
__device__ __forceinline__ void walk_sum(u64 s_first, u64* S, double& H, double& L) {
  u32 top = 0;
  walk_sum_run<V, KEEP, true>(s_first, S, H, L, top);
  if (wave_any_unreduced(top)) walk_sum_run<V, KEEP, false>(s_first, S, H, L, top);
}

// Inclusive scan over the wave of integer-valued doubles whose partial sums
// stay below 2^53 (exact in any order): the DPP pattern of wave_scan_mod, the
// moved bits reinterpreted as doubles (a lane with no source receives +0.0).
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_f64(double x) {
  return __longlong_as_double((long long)dpp64<CTRL, ROW_MASK>((u64)__double_as_longlong(x)));
}

__device__ __forceinline__ double wave_scan_f64(double x, int) {
  x += dpp_f64<0x111, 0xf>(x);  // row_shr:1
  x += dpp_f64<0x112, 0xf>(x);  // row_shr:2
  x += dpp_f64<0x114, 0xf>(x);  // row_shr:4
  x += dpp_f64<0x118, 0xf>(x);  // row_shr:8
  x += dpp_f64<0x142, 0xa>(x);  // row_bcast:15 into rows 1 and 3
  x += dpp_f64<0x143, 0xc>(x);  // row_bcast:31 into rows 2 and 3
  return x;
}


// Dispatch of one lane's outputs on the exponent: ladders unrolled for the
// common exponents when every index of the span is requested and the stores
// are suitably aligned, a generic ladder with predicated stores otherwise.  EK
// != 0: every instance of the launch has exponent EK; the caller passes fast
// only for 16-byte-aligned outputs, so that this path carries no second store
// sequence (the register budget of those kernels is tight), and other chunks
// take the EK ladder with predicated stores.  The general kernels' fast path
// takes any 8-byte-aligned output (store_chunk tests the alignment).
template <int WG, int V, int VAR, int MODE, int EK = 0, int AL = 1, class Msg>
__device__ __forceinline__ void outputs_for_e(const LaunchArgs& a, TileShared<WG, MODE>& sh,
                                              const Chain& C, const rsaprng_params& P,
                                              const Msg& msg, bool fast, u64 laneStart) {
  if constexpr (EK != 0) {
    if (fast)
      tile_outputs<WG, V, VAR, MODE, EK, true, AL, true>(a, sh, C, P, msg, laneStart);
    else
      tile_outputs<WG, V, VAR, MODE, EK, false>(a, sh, C, P, msg, laneStart);
  } else if (!fast) {
    tile_outputs<WG, V, VAR, MODE, 0, false>(a, sh, C, P, msg, laneStart);
  } else {
    switch (P.e) {
      case 1: tile_outputs<WG, V, VAR, MODE, 1, true>(a, sh, C, P, msg, laneStart); break;
      case 3: tile_outputs<WG, V, VAR, MODE, 3, true>(a, sh, C, P, msg, laneStart); break;
      case 5: tile_outputs<WG, V, VAR, MODE, 5, true>(a, sh, C, P, msg, laneStart); break;
      case 7: tile_outputs<WG, V, VAR, MODE, 7, true>(a, sh, C, P, msg, laneStart); break;
      case 17: tile_outputs<WG, V, VAR, MODE, 17, true>(a, sh, C, P, msg, laneStart); break;
      case 257: tile_outputs<WG, V, VAR, MODE, 257, true>(a, sh, C, P, msg, laneStart); break;
      case 65537: tile_outputs<WG, V, VAR, MODE, 65537, true>(a, sh, C, P, msg, laneStart); break;
      default: tile_outputs<WG, V, VAR, MODE, 0, true>(a, sh, C, P, msg, laneStart); break;
    }
  }
}

// Outputs of one wave chunk (64 V indices starting at chunkStart).  The fast
// path needs every index of the chunk requested; in the general kernels with
// V = 8 its stores take any 8-byte-aligned output (store_chunk), the pair
// stores of other V need 16-byte alignment, and so do the paths specialised
// to one exponent with AL = 1 (the kernels for launches of one exponent, V = 8
// or 16); with AL = -1 (the per-chain dispatch over exponents) they test it.
template <int WG, int V, int VAR, int MODE, int EK = 0, int AL = 1, class Msg>
__device__ __forceinline__ void chunk_outputs(const LaunchArgs& a, TileShared<WG, MODE>& sh,
                                              const Chain& C, const rsaprng_params& P,
                                              const Msg& msg, u64 chunkStart, u64 laneStart) {
  constexpr u64 CHUNK = 64ull * V;
  const u64 off_c = C.out_off + (chunkStart - C.k0);
  // 16-byte-aligned outputs (evaluated only for a full chunk)
  const auto a16 = [&] {
    return (!a.out_c || ((uintptr_t)(a.out_c + off_c) & 15) == 0) &&
           (!a.out_r || ((uintptr_t)(a.out_r + off_c) & 15) == 0);
  };
  const bool full = chunkStart >= C.k0 && chunkStart + (CHUNK - 1) <= C.last;
  if constexpr (EK != 0)
    outputs_for_e<WG, V, VAR, MODE, EK, AL>(a, sh, C, P, msg, full && (AL == -1 || a16()),
                                            laneStart);
  else
    outputs_for_e<WG, V, VAR, MODE, EK>(a, sh, C, P, msg,
                                        full && (MODE != kModeGenerate || V == 8 || a16()),
                                        laneStart);
}

// The same state from residue messages (b the residues of the message before
// the lane's first index, s_first its skip): m at the last index recombined by
// Garner (encryption with e = 1) and the skip after it.
template <int V>
__device__ __forceinline__ void chain_end_res(const LaunchArgs& a, const Chain& C,
                                              const rsaprng_params& P, u64 s_first, double bp,
                                              double bq, u64 laneStart) {
  if ((C.flags & kChainWriteEnd) && laneStart <= C.last && C.last - laneStart < (u64)V) {
    double H = 0.0, L = 0.0;
    u64 s = s_first, s_last = 0;
#pragma unroll
    for (int i = 0; i < V; ++i) {
      if (i) s = lcg_next(s);
      if (laneStart + i <= C.last) {
        H += (double)hi32(s);
        L += (double)lo32(s);
        s_last = s;
      }
    }
    const double mp = reduce_res(bp + (fold_p(H, P) + L), P.pd, P.pinv);
    const double mq = reduce_res(bq + (fold_q(H, P) + L), P.qd, P.qinv);
    double cd;
    ChainState cs;
    cs.m_prev = garner(mp, mq, P.pd, P.qd, P.pinv, P.qinv, P.gp_lo, P.gp_hi, P.gp_quo, P.q, cd);
    cs.s_at = lcg_next(s_last);
    a.state[C.slot] = cs;
  }
}

// The exact state, walking from the lane's first skip.
template <int V>
__device__ __forceinline__ void chain_end_walk(const LaunchArgs& a, const Chain& C, u64 n,
                                               u64 pre, u64 s_first, u64 laneStart) {
  if ((C.flags & kChainWriteEnd) && laneStart <= C.last && C.last - laneStart < (u64)V) {
    u64 s = s_first, x = 0, s_last = 0;
#pragma unroll
    for (int i = 0; i < V; ++i) {
      if (i) s = lcg_next(s);
      if (laneStart + i <= C.last) {
        x = addmod(x, skip_mod_n(s, n), n);
        s_last = s;
      }
    }
    ChainState cs;
    cs.m_prev = addmod(pre, x, n);
    cs.s_at = lcg_next(s_last);
    a.state[C.slot] = cs;
  }
}

// Chain-end state for a continued request: the lane holding the last index.
template <int V>
__device__ __forceinline__ void chain_end(const LaunchArgs& a, const Chain& C, u64 n, u64 pre,
                                          const u64 (&X)[V], u64 s_first, u64 laneStart) {
  if ((C.flags & kChainWriteEnd) && laneStart <= C.last && C.last - laneStart < (u64)V) {
    u64 m_end = 0;
    u64 ss = s_first;
#pragma unroll
    for (int i = 0; i < V; ++i) {
      if (laneStart + i == C.last) m_end = addmod(pre, X[i], n);
      if (laneStart + i < C.last) ss = lcg_next(ss);
    }
    ChainState cs;
    cs.m_prev = m_end;
    cs.s_at = lcg_next(ss);
    a.state[C.slot] = cs;
  }
}

// Exponent dispatch of the tile kernels: EK > 0, the kernel's paths are
// specialised to that exponent; EK = kEKPerChain, each chain (or tile) takes
// the path specialised to its own exponent (the common ones; any other, and
// dual-exponent instances, take the general path, EK = 0).
constexpr int kEKPerChain = -1;

// Two passes: each wave owns R consecutive chunks of 64 V indices of the tile
// (T = WG V R) and processes them one after the other; the message before a
// chunk comes from k_scan (for CRT as its two residues) and its start skip
// from the tile's skip, a^(64 V q) for the chunk (wave-uniform) and a^(V lane),
// so waves never wait on each other.  EK as for k_gen3: with EK != 0 the
// fast path takes any 8-byte-aligned output (AL = -1).
template <int WG, int V, int R, int VAR, int MODE, int EK>
__device__ __forceinline__ void tile2(const LaunchArgs& a, TileShared<WG, MODE>& sh, u32 t,
                                      u64 pl, int lane, u32 wave) {
  constexpr int NW = WG / 64;
  constexpr int CH = NW * R;  // chunks per tile
  constexpr u64 T = (u64)WG * V * R;
  constexpr u64 CHUNK = 64ull * V;
  const u32 c = cst(a.tile_chain)[t];
  const Chain C = load_cst(a.chain + c);
  const rsaprng_params P = load_cst(a.inst + C.inst);
  const u64 n = P.n;
  const u64 tileStart = C.S + (u64)(t - C.first) * T;
  const u64 s_tile = cst(a.s_tile)[t];
  const u32 q0 = wave * R;  // first chunk of this wave
  const bool any_out = tileStart + (T - 1) >= C.k0;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const u64 chunkStart = tileStart + (u64)(q0 + r) * CHUNK;
    const u64 laneStart = chunkStart + (u64)lane * V;
    const bool outs = MODE == kModeConsume ? any_out : chunkStart + (CHUNK - 1) >= C.k0;
    if (!outs && !(C.flags & kChainWriteEnd)) continue;
    // the message before the chunk (CRT: its residues mod p and q), used
    // after the walk and the scans
    const u64 q = (u64)t * CH + q0 + r;
    const u64 E1 = cst(a.excl)[q];
    const u64 E2 = VAR == kVariantCrt ? cst(a.agg)[q] : 0;
    // the chunk's first skip (wave-uniform, scalar arithmetic), then each lane's
    const u64 s_chunk = mulmod_q(s_tile, cst(a.powv)[(u64)(q0 + r) * 64]);
    const u64 s_first = mulmod_q(s_chunk, pl);
    if constexpr (VAR == kVariantCrt) {
      // lane totals as residues up to multiples of p and q, scanned in exact
      // binary64 arithmetic: |tp| < 2^33 (Ht < 2^35, Lt < 2^32), so the
      // partial sums stay below 2^39 and the sums formed for reduce_res
      // below 2^40
      u64 S[V];
      double Ht, Lt;
      walk_sum<V, true>(s_first, S, Ht, Lt);
      const double tp = fold_p(Ht, P) + Lt;
      const double tq = fold_q(Ht, P) + Lt;
      const double ip = wave_scan_f64(tp, lane);
      const double iq = wave_scan_f64(tq, lane);
      const double Ep = __longlong_as_double((long long)E2);
      const double Eq = __longlong_as_double((long long)E1);
      const double bp = reduce_res(Ep + (ip - tp), P.pd, P.pinv);
      const double bq = reduce_res(Eq + (iq - tq), P.qd, P.qinv);
      const MsgRes<V> msg{S, bp, bq};
      if (outs) chunk_outputs<WG, V, VAR, MODE, EK, -1>(a, sh, C, P, msg, chunkStart, laneStart);
      chain_end_res<V>(a, C, P, s_first, bp, bq, laneStart);
    } else {
      u64 X[V];
      const u64 x = walk<V>(s_first, n, X);
      const u64 incl = wave_scan_mod(x, n);
      const u64 pre = addmod(E1, submod(incl, x, n), n);
      const MsgExact<V> msg{pre, n, X};
      if (outs) chunk_outputs<WG, V, VAR, MODE>(a, sh, C, P, msg, chunkStart, laneStart);
      chain_end<V>(a, C, n, pre, X, s_first, laneStart);
    }
  }
  if constexpr (MODE == kModeConsume) {
    if (any_out) consume_flush<WG>(a, sh, C.slot);
  }
}

template <int WG, int V, int R, int VAR, int MODE, int EK = 0>
__global__ __launch_bounds__(WG) __attribute__((amdgpu_waves_per_eu(EK != 0 ? 4 : 1)))
void k_gen2(LaunchArgs a) {
  static_assert(EK == 0 || (MODE == kModeGenerate && VAR == kVariantCrt),
                "specialised paths: CRT generate");
  __shared__ TileShared<WG, MODE> sh;
  const int lane = threadIdx.x & 63;
  const u32 wave = uniform(threadIdx.x >> 6);
  const u64 pl = a.powv[lane];  // a^(V lane)
  if constexpr (MODE == kModeConsume) {
    for (int b = threadIdx.x; b < 1024; b += WG) sh.hist[b] = 0;
    for (int j = 0; j < 7; ++j) sh.acc[j * WG + threadIdx.x] = 0;
    __syncthreads();
  }
  for (u32 t = a.tile0 + blockIdx.x; t < a.ntiles; t += gridDim.x) {
    if constexpr (EK == kEKPerChain) {
      const u32 inst = cst(&a.chain[cst(a.tile_chain)[t]].inst)[0];
      switch (cst(&a.inst[inst].e)[0]) {
        case 3: tile2<WG, V, R, VAR, MODE, 3>(a, sh, t, pl, lane, wave); break;
        case 5: tile2<WG, V, R, VAR, MODE, 5>(a, sh, t, pl, lane, wave); break;
        case 7: tile2<WG, V, R, VAR, MODE, 7>(a, sh, t, pl, lane, wave); break;
        case 17: tile2<WG, V, R, VAR, MODE, 17>(a, sh, t, pl, lane, wave); break;
        case 257: tile2<WG, V, R, VAR, MODE, 257>(a, sh, t, pl, lane, wave); break;
        case 65537: tile2<WG, V, R, VAR, MODE, 65537>(a, sh, t, pl, lane, wave); break;
        default: tile2<WG, V, R, VAR, MODE, 0>(a, sh, t, pl, lane, wave); break;
      }
    } else {
      tile2<WG, V, R, VAR, MODE, EK>(a, sh, t, pl, lane, wave);
    }
  }
}

// One pass: tiles of T = WG V claimed from an atomic queue; the wave totals go
// through LDS and the message before the tile comes from the look-back.
template <int WG, int V, int VAR, int MODE>
__global__ __launch_bounds__(WG) void k_gen1(LaunchArgs a) {
  constexpr int NW = WG / 64;
  constexpr u64 T = (u64)WG * V;
  __shared__ TileShared<WG, MODE> sh;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const u64 my_powv = a.powv[threadIdx.x];
  if constexpr (MODE == kModeConsume) {
    for (int b = threadIdx.x; b < 1024; b += WG) sh.hist[b] = 0;
    for (int j = 0; j < 7; ++j) sh.acc[j * WG + threadIdx.x] = 0;
  }
  const u32 tag = a.ctl->epoch;
  for (;;) {
    if (threadIdx.x == 0) sh.tile = atomicAdd(&a.ctl->counter, 1u);
    __syncthreads();
    const u32 t = uniform(sh.tile);
    if (t >= a.ntiles) break;
    const u32 c = uniform(a.tile_chain[t]);
    const Chain C = a.chain[c];
    const rsaprng_params P = a.inst[C.inst];
    const u64 n = P.n;
    const u32 j = t - C.first;
    const u64 tileStart = C.S + (u64)j * T;
    const u64 s_tile = mulmod_q(a.cstart[c].s_S, a.at[j]);
    const u64 laneStart = tileStart + (u64)threadIdx.x * V;
    u64 X[V];
    const u64 s_first = mulmod_q(s_tile, my_powv);
    const u64 x = walk<V>(s_first, n, X);
    const u64 incl = wave_scan_mod(x, n);
    if (lane == 63) sh.wave_tot[wave] = incl;
    __syncthreads();
    u64 wave_off = 0, agg = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w) {
      const u64 v = sh.wave_tot[w];
      if (w < wave) wave_off = addmod(wave_off, v, n);
      agg = addmod(agg, v, n);
    }
    if (wave == 0) {
      u64 Ew;
      if (j == 0) {
        Ew = a.cstart[c].m_base;
      } else {
        if (lane == 0) publish(a.lb + 4ull * t, tag, agg);
        Ew = look_back(a, t, C.first, tag, n, lane);
      }
      if (lane == 0) {
        publish(a.lb + 4ull * t + 2, tag, addmod(Ew, agg, n));
        sh.pre = Ew;
      }
    }
    __syncthreads();
    const u64 pre = addmod(addmod(sh.pre, wave_off, n), submod(incl, x, n), n);
    if (tileStart + (T - 1) >= C.k0) {
      // the fast path is decided per tile here so every wave takes the same barriers
      const u64 off_t = C.out_off + (tileStart - C.k0);
      const bool fast = tileStart >= C.k0 && tileStart + (T - 1) <= C.last &&
                        (MODE == kModeConsume || V == 8 ||
                         ((!a.out_c || ((uintptr_t)(a.out_c + off_t) & 15) == 0) &&
                          (!a.out_r || ((uintptr_t)(a.out_r + off_t) & 15) == 0)));
      outputs_for_e<WG, V, VAR, MODE>(a, sh, C, P, MsgExact<V>{pre, n, X}, fast, laneStart);
      if constexpr (MODE == kModeConsume) consume_flush<WG>(a, sh, C.slot);
    }
    chain_end<V>(a, C, n, pre, X, s_first, laneStart);
    __syncthreads();
  }
}

// Chain-serial: one work-group per chain walks it in steps of T = WG V R
// indices (wave w takes chunks w R .. w R + R - 1 of 64 V indices, so its R
// >= 2 walks are independent), carrying the message before the step from one step
// to the next -- as residues mod p and q for the CRT variant, exactly mod n
// for the Montgomery variant.  The waves exchange their totals through LDS
// once per step (double-buffered by step parity: one barrier per step).  The
// output pass walks each chunk again from its first skip instead of keeping
// R V skips across the barrier, except on the paths specialised to one
// exponent (EK != 0, generate mode): with a single ladder in the loop the
// skips fit the register budget of four waves per SIMD (which the transpose
// buffers' LDS caps residency at anyway), so they are kept.  Steps before the
// chain's first requested index only walk.  No prefix pass is needed.
//
// chain3 runs one chain; k_gen3 loops over the chains.  EK > 0: every chain
// of the launch has exponent EK (outputs 16-byte aligned for the fast path,
// AL = 1).  EK = kEKPerChain: each chain dispatches on its exponent to the
// path specialised to it (the common exponents; any other, and the
// dual-exponent instances, take the general path), with the fast path taking
// any 8-byte-aligned output (AL = -1).  Each path is its own loop nest, so the
// kernel's register budget is the largest one's, not their sum.

template <int WG, int V, int R, int VAR, int MODE, int EK, int AL>
__device__ __forceinline__ void chain3(const LaunchArgs& a, TileShared<WG, MODE>& sh,
                                       double2 (&xch)[2][WG / 64], u32 c, const u64 (&pv)[R],
                                       u64 aT, int lane, u32 wave) {
  constexpr int NW = WG / 64;
  constexpr u64 T = (u64)WG * V * R;
  constexpr u64 CHUNK = 64ull * V;
  const Chain C = load_cst(a.chain + c);
  const rsaprng_params P = load_cst(a.inst + C.inst);
  const ChainStart cs0 = load_cst(a.cstart + c);
  const u64 n = P.n;
  // the chain ends at the request's last index or at the end of its 2^20 block
  const u64 clast = C.last < (C.S | (kBlock - 1)) ? C.last : (C.S | (kBlock - 1));
  u64 s_step = cs0.s_S;       // skip at the step's first index
  double cp = 0.0, cq = 0.0;  // CRT carry: residues of the message before the step
  u64 cm = 0;                 // Montgomery carry: the message before the step
  if constexpr (VAR == kVariantCrt) {
    cp = cs0.rp;  // residues of m_base, from the chain setup
    cq = cs0.rq;
  } else {
    cm = cs0.m_base;
  }
  for (u32 step = 0;; ++step) {
    const u64 base = C.S + (u64)step * T;
    const bool step_out = base + (T - 1) >= C.k0;  // uniform over the work-group
    const int par = step & 1;
    u64 sf[R];
#pragma unroll
    for (int r = 0; r < R; ++r) sf[r] = mulmod_q(s_step, pv[r]);
    if constexpr (VAR == kVariantCrt) {
      // per chunk: lane totals as residues, exclusive lane prefix plus the
      // totals of the wave's earlier chunks
      double ep[R], eq[R];
      double wp = 0.0, wq = 0.0;
      constexpr bool kKeep = EK != 0;
      u64 S[R][kKeep ? V : 1];  // the kept skips of each chunk
#pragma unroll
      for (int r = 0; r < R; ++r) {
        double Ht, Lt;
        walk_sum<V, kKeep>(sf[r], S[r], Ht, Lt);
        // unreduced: |tp| < 2^33, so the lane prefixes stay below 2^39, the
        // wave totals below 2^41 and their sums over the work-group below 2^45
        const double tp = fold_p(Ht, P) + Lt;
        const double tq = fold_q(Ht, P) + Lt;
        const double ip = wave_scan_f64(tp, lane);
        const double iq = wave_scan_f64(tq, lane);
        ep[r] = wp + (ip - tp);
        eq[r] = wq + (iq - tq);
        wp += lane_value_f64(ip, 63);
        wq += lane_value_f64(iq, 63);
      }
      if (lane == 63) xch[par][wave] = make_double2(wp, wq);
      __syncthreads();
      double op = 0.0, oq = 0.0, Tp = 0.0, Tq = 0.0;
      // the wave index re-read each step: otherwise the NW factors below are
      // hoisted out of the chain loop and held in scalar registers
      u32 wv = wave;
      asm volatile("" : "+s"(wv));
#pragma unroll
      for (int w = 0; w < NW; ++w) {
        const double2 v = xch[par][w];
        // a wave-uniform 1 for the waves before this one: one fma instead of
        // a select and an add (integers below 2^53, every step exact)
        const double f = w < (int)wv ? 1.0 : 0.0;
        op = __fma_rn(f, v.x, op);
        oq = __fma_rn(f, v.y, oq);
        Tp += v.x;
        Tq += v.y;
      }
      if (step_out) {
        if constexpr (kKeep) {
          // unrolled by instantiation: the kept skips are indexed statically
          static_for<0, R>([&](auto rc) {
            constexpr int r = decltype(rc)::value;
            const u64 chunkStart = base + ((u64)wave * R + r) * CHUNK;
            const u64 laneStart = chunkStart + (u64)lane * V;
            const double bp = reduce_res(cp + op + ep[r], P.pd, P.pinv);
            const double bq = reduce_res(cq + oq + eq[r], P.qd, P.qinv);
            if (chunkStart + (CHUNK - 1) >= C.k0 && chunkStart <= clast) {
              const MsgRes<V> msg{S[r], bp, bq};
              chunk_outputs<WG, V, VAR, MODE, EK, AL>(a, sh, C, P, msg, chunkStart, laneStart);
            }
            chain_end_res<V>(a, C, P, sf[r], bp, bq, laneStart);
          });
        } else {
#pragma unroll
          for (int r = 0; r < R; ++r) {
            const u64 chunkStart = base + ((u64)wave * R + r) * CHUNK;
            const u64 laneStart = chunkStart + (u64)lane * V;
            const double bp = reduce_res(cp + op + ep[r], P.pd, P.pinv);
            const double bq = reduce_res(cq + oq + eq[r], P.qd, P.qinv);
            const bool chunk_out = MODE == kModeConsume ||
                                   (chunkStart + (CHUNK - 1) >= C.k0 && chunkStart <= clast);
            const MsgResWalk<V> msg{sf[r], bp, bq};
            if (chunk_out) chunk_outputs<WG, V, VAR, MODE>(a, sh, C, P, msg, chunkStart, laneStart);
            chain_end_res<V>(a, C, P, sf[r], bp, bq, laneStart);
          }
        }
      }
      cp = reduce_res(cp + Tp, P.pd, P.pinv);
      cq = reduce_res(cq + Tq, P.qd, P.qinv);
    } else {
      u64 ex[R];
      u64 wt = 0;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        u64 X[V];
        const u64 x = walk<V>(sf[r], n, X);
        const u64 incl = wave_scan_mod(x, n);
        ex[r] = addmod(wt, submod(incl, x, n), n);
        wt = addmod(wt, lane_value(incl, 63), n);
      }
      if (lane == 63) xch[par][wave].x = __longlong_as_double((long long)wt);
      __syncthreads();
      u64 off = 0, tot = 0;
#pragma unroll
      for (int w = 0; w < NW; ++w) {
        const u64 v = (u64)__double_as_longlong(xch[par][w].x);
        if (w < (int)wave) off = addmod(off, v, n);
        tot = addmod(tot, v, n);
      }
      if (step_out) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const u64 chunkStart = base + ((u64)wave * R + r) * CHUNK;
          const u64 laneStart = chunkStart + (u64)lane * V;
          const u64 pre = addmod(addmod(cm, off, n), ex[r], n);
          const MsgExactWalk<V> msg{pre, n, sf[r]};
          const bool chunk_out = MODE == kModeConsume ||
                                 (chunkStart + (CHUNK - 1) >= C.k0 && chunkStart <= clast);
          if (chunk_out) chunk_outputs<WG, V, VAR, MODE>(a, sh, C, P, msg, chunkStart, laneStart);
          chain_end_walk<V>(a, C, n, pre, sf[r], laneStart);
        }
      }
      cm = addmod(cm, tot, n);
    }
    if constexpr (MODE == kModeBattery) {
      if (step_out) msb_step<WG>(a, sh, base, (u32)T, C.k0, C.last, blockIdx.x);
      // a step that ends a collision trial whose indices were all requested
      // (T divides 2^14, so steps never straddle a trial)
      const u64 end = base + T;
      if ((end & ((1ull << kTrialLog2) - 1)) == 0 && end - (1ull << kTrialLog2) >= C.k0 &&
          end - 1 <= C.last)
        trial_flush<WG>(a, sh);
    }
    if (clast - base < T) break;
    s_step = mulmod_q(s_step, aT);
  }
  if constexpr (MODE == kModeConsume) consume_flush<WG>(a, sh, C.slot);
  if constexpr (MODE == kModeBattery) battery_flush<WG>(a, sh);
}

template <int WG, int V, int R, int VAR, int MODE, int EK = 0>
__global__ __launch_bounds__(WG) __attribute__((amdgpu_waves_per_eu(EK != 0 ? 4 : 1)))
void k_gen3(LaunchArgs a) {
  static_assert(EK == 0 || ((MODE == kModeGenerate || MODE == kModeConsume) && VAR == kVariantCrt),
                "specialised paths: CRT generate and consume");
  constexpr int NW = WG / 64;
  __shared__ TileShared<WG, MODE> sh;
  __shared__ double2 xch[2][NW];  // wave totals: residues (CRT) or the u64 bits in .x
  const int lane = threadIdx.x & 63;
  const u32 wave = uniform(threadIdx.x >> 6);
  u64 pv[R];  // a^(offset of the lane's first index in each of its chunks)
#pragma unroll
  for (int r = 0; r < R; ++r) pv[r] = a.powv[((u64)wave * R + r) * 64 + lane];
  const u64 aT = load_cst(a.at + 1);  // a^T mod Q
  if constexpr (MODE == kModeConsume) {
    for (int b = threadIdx.x; b < 1024; b += WG) sh.hist[b] = 0;
    for (int j = 0; j < 7; ++j) sh.acc[j * WG + threadIdx.x] = 0;
    __syncthreads();
  }
  if constexpr (MODE == kModeBattery) {
    for (int i = threadIdx.x; i < kUrnWords; i += WG) sh.urn[i] = 0;
    for (int i = threadIdx.x; i < kBatLds; i += WG) sh.bh[i] = 0;
    __syncthreads();
  }
  for (u32 c = blockIdx.x; c < a.nchain; c += gridDim.x) {
    if constexpr (EK == kEKPerChain) {
      const u32 inst = cst(&a.chain[c].inst)[0];
      switch (cst(&a.inst[inst].e)[0]) {
        case 3: chain3<WG, V, R, VAR, MODE, 3, -1>(a, sh, xch, c, pv, aT, lane, wave); break;
        case 5: chain3<WG, V, R, VAR, MODE, 5, -1>(a, sh, xch, c, pv, aT, lane, wave); break;
        case 7: chain3<WG, V, R, VAR, MODE, 7, -1>(a, sh, xch, c, pv, aT, lane, wave); break;
        case 17: chain3<WG, V, R, VAR, MODE, 17, -1>(a, sh, xch, c, pv, aT, lane, wave); break;
        case 257: chain3<WG, V, R, VAR, MODE, 257, -1>(a, sh, xch, c, pv, aT, lane, wave); break;
        case 65537:
          chain3<WG, V, R, VAR, MODE, 65537, -1>(a, sh, xch, c, pv, aT, lane, wave);
          break;
        default: chain3<WG, V, R, VAR, MODE, 0, 1>(a, sh, xch, c, pv, aT, lane, wave); break;
      }
    } else {
      chain3<WG, V, R, VAR, MODE, EK, 1>(a, sh, xch, c, pv, aT, lane, wave);
    }
  }
}

template <int WG, int V, int R, int VAR, int MODE, int EK = 0>
static int launch3(const LaunchArgs& a, int grid, void* stream, int* occ) {
  if (occ) {
    int blocks = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_gen3<WG, V, R, VAR, MODE, EK>, WG,
                                                     0) != hipSuccess)
      blocks = 1;
    *occ = blocks > 0 ? blocks : 1;
    return RSAPRNG_OK;
  }
  hipLaunchKernelGGL((k_gen3<WG, V, R, VAR, MODE, EK>), dim3(grid), dim3(WG), 0,
                     (hipStream_t)stream, a);
  return hipGetLastError() == hipSuccess ? RSAPRNG_OK : RSAPRNG_E_HIP;
}

template <int WG, int V, int R, int VAR, int MODE, int EK = 0>
static int launch2(const LaunchArgs& a, int grid, void* stream, int* occ) {
  if (occ) {
    int blocks = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_gen2<WG, V, R, VAR, MODE, EK>, WG,
                                                     0) != hipSuccess)
      blocks = 1;
    *occ = blocks > 0 ? blocks : 1;
    return RSAPRNG_OK;
  }
  hipLaunchKernelGGL((k_gen2<WG, V, R, VAR, MODE, EK>), dim3(grid), dim3(WG), 0,
                     (hipStream_t)stream, a);
  return hipGetLastError() == hipSuccess ? RSAPRNG_OK : RSAPRNG_E_HIP;
}

template <int WG, int V, int VAR, int MODE>
static int launch1(const LaunchArgs& a, int grid, void* stream, int* occ) {
  if (occ) {
    int blocks = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_gen1<WG, V, VAR, MODE>, WG, 0) !=
        hipSuccess)
      blocks = 1;
    *occ = blocks > 0 ? blocks : 1;
    return RSAPRNG_OK;
  }
  hipLaunchKernelGGL((k_gen1<WG, V, VAR, MODE>), dim3(grid), dim3(WG), 0, (hipStream_t)stream, a);
  return hipGetLastError() == hipSuccess ? RSAPRNG_OK : RSAPRNG_E_HIP;
}

// Launcher and occupancy query for every shape of one (variant, mode).
template <int VAR, int MODE>
int launch_family(const KernelShape& s, const LaunchArgs& a, void* stream, int* occ) {
  if constexpr (MODE == kModeBattery) {  // the battery needs a work-group per chain
    if (s.prefix != kPrefixSerial) return RSAPRNG_E_ARG;
    if (s.wg == 256 && s.v == 8 && s.r == 2) return launch3<256, 8, 2, VAR, MODE>(a, s.grid, stream, occ);
    if (s.wg == 256 && s.v == 8 && s.r == 4) return launch3<256, 8, 4, VAR, MODE>(a, s.grid, stream, occ);
    if (s.wg == 512 && s.v == 8 && s.r == 2) return launch3<512, 8, 2, VAR, MODE>(a, s.grid, stream, occ);
    return RSAPRNG_E_ARG;
  } else {
    if (s.prefix == kPrefixTwoPass) {
      if (s.wg == 256 && s.v == 8 && s.r == 1) return launch2<256, 8, 1, VAR, MODE>(a, s.grid, stream, occ);
      if (s.wg == 256 && s.v == 8 && s.r == 2) return launch2<256, 8, 2, VAR, MODE>(a, s.grid, stream, occ);
      if (s.wg == 256 && s.v == 8 && s.r == 4) return launch2<256, 8, 4, VAR, MODE>(a, s.grid, stream, occ);
      if (s.wg == 512 && s.v == 8 && s.r == 2) return launch2<512, 8, 2, VAR, MODE>(a, s.grid, stream, occ);
      if constexpr (MODE == kModeGenerate && VAR == kVariantCrt) {
        // 16 indices per lane: the kernel specialised to the launch's (or the
        // exponent class's) exponent, else each tile takes its own
        if (s.wg == 256 && s.v == 16 && s.r == 2) {
          switch (s.e) {
            case 3: return launch2<256, 16, 2, VAR, MODE, 3>(a, s.grid, stream, occ);
            case 5: return launch2<256, 16, 2, VAR, MODE, 5>(a, s.grid, stream, occ);
            case 7: return launch2<256, 16, 2, VAR, MODE, 7>(a, s.grid, stream, occ);
            case 17: return launch2<256, 16, 2, VAR, MODE, 17>(a, s.grid, stream, occ);
            case 257: return launch2<256, 16, 2, VAR, MODE, 257>(a, s.grid, stream, occ);
            case 65537: return launch2<256, 16, 2, VAR, MODE, 65537>(a, s.grid, stream, occ);
            default: return launch2<256, 16, 2, VAR, MODE, kEKPerChain>(a, s.grid, stream, occ);
          }
        }
      }
      return RSAPRNG_E_ARG;
    }
    if (s.prefix == kPrefixSerial) {
      if constexpr (MODE == kModeConsume && VAR == kVariantCrt) {
        if (s.wg == 256 && s.v == 8 && s.r == 2) return launch3<256, 8, 2, VAR, MODE, kEKPerChain>(a, s.grid, stream, occ);
        // launches of one exponent with 16 indices per lane: kernels specialised
        // to it (the per-chain dispatch at that shape would spill)
        if (s.wg == 256 && s.v == 16 && s.r == 1) {
          switch (s.e) {
            case 3: return launch3<256, 16, 1, VAR, MODE, 3>(a, s.grid, stream, occ);
            case 5: return launch3<256, 16, 1, VAR, MODE, 5>(a, s.grid, stream, occ);
            case 7: return launch3<256, 16, 1, VAR, MODE, 7>(a, s.grid, stream, occ);
            case 17: return launch3<256, 16, 1, VAR, MODE, 17>(a, s.grid, stream, occ);
            case 257: return launch3<256, 16, 1, VAR, MODE, 257>(a, s.grid, stream, occ);
            case 65537: return launch3<256, 16, 1, VAR, MODE, 65537>(a, s.grid, stream, occ);
            default: return RSAPRNG_E_ARG;
          }
        }
      }
      if constexpr (MODE == kModeGenerate && VAR == kVariantCrt) {
        // every instance of the launch has e = 3: the kernels specialised to
        // it; otherwise each chain takes the path specialised to its own
        // exponent (not for four chunks per wave, whose kept skips would spill)
        if (s.e == 3) {
          if (s.wg == 256 && s.v == 8 && s.r == 2) return launch3<256, 8, 2, VAR, MODE, 3>(a, s.grid, stream, occ);
          if (s.wg == 512 && s.v == 8 && s.r == 2) return launch3<512, 8, 2, VAR, MODE, 3>(a, s.grid, stream, occ);
          if (s.wg == 256 && s.v == 16 && s.r == 1) return launch3<256, 16, 1, VAR, MODE, 3>(a, s.grid, stream, occ);
          if (s.wg == 512 && s.v == 16 && s.r == 1) return launch3<512, 16, 1, VAR, MODE, 3>(a, s.grid, stream, occ);
        }
        if (s.wg == 256 && s.v == 8 && s.r == 2) return launch3<256, 8, 2, VAR, MODE, kEKPerChain>(a, s.grid, stream, occ);
        if (s.wg == 512 && s.v == 8 && s.r == 2) return launch3<512, 8, 2, VAR, MODE, kEKPerChain>(a, s.grid, stream, occ);
      }
      if (s.wg == 256 && s.v == 8 && s.r == 2) return launch3<256, 8, 2, VAR, MODE>(a, s.grid, stream, occ);
      if (s.wg == 256 && s.v == 8 && s.r == 4) return launch3<256, 8, 4, VAR, MODE>(a, s.grid, stream, occ);
      if (s.wg == 512 && s.v == 8 && s.r == 2) return launch3<512, 8, 2, VAR, MODE>(a, s.grid, stream, occ);
      return RSAPRNG_E_ARG;
    }
    if (s.r != 1) return RSAPRNG_E_ARG;
    if (s.wg == 256 && s.v == 8) return launch1<256, 8, VAR, MODE>(a, s.grid, stream, occ);
    if (s.wg == 512 && s.v == 8) return launch1<512, 8, VAR, MODE>(a, s.grid, stream, occ);
    if (s.wg == 256 && s.v == 16) return launch1<256, 16, VAR, MODE>(a, s.grid, stream, occ);
    return RSAPRNG_E_ARG;
  }
}

}  // namespace rsaprng
