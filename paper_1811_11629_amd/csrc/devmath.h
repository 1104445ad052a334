// Device arithmetic for gfx950: the skip recurrence mod Q = 2^63 - 25, the
// message update mod n, 64-bit Montgomery multiplication from 32-bit limbs,
// and the CRT form of the exponentiation with residues held in binary64.
//
// On gfx950 v_mad_u64_u32, v_mul_lo_u32 and v_mul_hi_u32 issue at the full
// VALU rate, as do binary64 fma/mul/rndne (the throughput probes of
// rsaprng_probe measure 0.90-0.96 of 256 CUs x 64 lanes x 2.4 GHz for each of
// these classes on an MI355X), so the 64-bit products below are
// written as 32x32->64 multiply-adds that the compiler maps onto
// v_mad_u64_u32; every bound on an intermediate is stated where it is formed.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rsaprng {

typedef uint64_t u64;
typedef uint32_t u32;

constexpr u64 kQ = 9223372036854775783ull;  // 2^63 - 25 (Implementation section)
constexpr u64 kA = 2307085864ull;           // skip multiplier
constexpr u64 kMask63 = 0x7fffffffffffffffull;

__device__ __forceinline__ u32 lo32(u64 x) { return (u32)x; }
__device__ __forceinline__ u32 hi32(u64 x) { return (u32)(x >> 32); }
__device__ __forceinline__ u64 mad32(u32 a, u32 b, u64 c) { return (u64)a * b + c; }

// Reduce r < 2^63 + 2^40 modulo Q, using 2^63 = 25 (mod Q): r >= Q exactly when
// r + 25 >= 2^63, and then r - Q = (r + 25) - 2^63.
__device__ __forceinline__ u64 reduce_q_small(u64 r) {
  u64 r2 = r + 25;
  return (r2 >> 63) ? (r2 & kMask63) : r;
}

// One skip step s -> a s mod Q (eq. congruentialgenerator1) without the final
// reduction.  a < 2^32 and s < 2^63 + 2^37, so a s = t1 2^32 + lo32(t0) with
// t1 < 2^63 (hi32(s) <= 2^31 + 2^5, a < 2^31.11); splitting a s as H 2^63 + L
// gives a s = 25 H + L (mod Q) with H < 2^32, and r = 25 H + L < 2^63 + 2^37 is
// a valid input again.  Three full-rate v_mad_u64_u32.  H is taken with an
// explicit funnel shift (bits 31..62 of t1): written as a shift and a
// truncation, the compiler widened it and added a zero term.
// r >= Q needs hi32(r) >= kHiUnreduced, so a run of such steps whose largest
// hi32 stays below it consists of reduced skips only (about one step in 2^31
// fails the test; the callers then redo the run with lcg_next).
constexpr u32 kHiUnreduced = 0x7fffffffu;  // hi32(Q)
__device__ __forceinline__ u64 lcg_lazy(u64 s) {
  u64 t0 = (u64)(u32)kA * lo32(s);
  u64 t1 = mad32((u32)kA, hi32(s), hi32(t0));
  const u32 H = __builtin_amdgcn_alignbit(hi32(t1), lo32(t1), 31);
  u64 L = ((t1 & 0x7fffffffull) << 32) | lo32(t0);
  return mad32(H, 25u, L);
}

// One skip step, reduced: a s mod Q in [0, Q).
__device__ __forceinline__ u64 lcg_next(u64 s) { return reduce_q_small(lcg_lazy(s)); }

// True when some lane of the wave has top >= kHiUnreduced: its run of lazy
// steps may hold a value >= Q (a wave-uniform test, so that the exact redo is
// a branch the wave takes together).
__device__ __forceinline__ bool wave_any_unreduced(u32 top) {
  return __builtin_expect(__builtin_amdgcn_ballot_w64(top >= kHiUnreduced) != 0, 0);
}

// One skip step of a lane's walk: lazy (lcg_lazy, the largest hi32 kept in
// top) or reduced.
template <bool LAZY>
__device__ __forceinline__ u64 walk_step(u64 s, u32& top) {
  if constexpr (LAZY) {
    const u64 r = lcg_lazy(s);
    top = max(top, hi32(r));
    return r;
  } else {
    return lcg_next(s);
  }
}

// Full 64x64 -> 128 product.
__device__ __forceinline__ void mul_wide(u64 x, u64 y, u64& lo, u64& hi) {
  u64 p00 = (u64)lo32(x) * lo32(y);
  u64 p01 = mad32(lo32(x), hi32(y), hi32(p00));
  u64 p10 = mad32(hi32(x), lo32(y), lo32(p01));
  hi = mad32(hi32(x), hi32(y), hi32(p01)) + hi32(p10);  // x y < 2^128: no wrap
  lo = ((u64)lo32(p10) << 32) | lo32(p00);
}

// x y mod Q for x, y < Q (jumps).  P = H 2^63 + L = 25 H + L; 25 H < 2^68 is
// folded once more the same way.
__device__ __forceinline__ u64 mulmod_q(u64 x, u64 y) {
  u64 lo, hi;
  mul_wide(x, y, lo, hi);
  u64 H = (hi << 1) | (lo >> 63);               // < 2^63
  u64 L = lo & kMask63;
  u64 u0 = mad32(lo32(H), 25u, L);              // < 2^37 + 2^63
  u64 u1 = mad32(hi32(H), 25u, hi32(u0));       // V = u1 2^32 + lo32(u0) < 2^69
  u32 H2 = (u32)(u1 >> 31);
  u64 L2 = ((u1 & 0x7fffffffull) << 32) | lo32(u0);
  return reduce_q_small(mad32(H2, 25u, L2));    // < 2^63 + 2^11
}

// (x + y) mod n for x, y < n < 2^64 (the message update m_k = m_{k-1} + s_k).
__device__ __forceinline__ u64 addmod(u64 x, u64 y, u64 n) {
  u64 s = x + y;
  bool carry = s < x;
  return (carry || s >= n) ? s - n : s;
}

// A skip s < Q < 2^63 <= 2n (n >= 2^62) reduced to [0, n) with one subtraction.
__device__ __forceinline__ u64 skip_mod_n(u64 s, u64 n) { return s >= n ? s - n : s; }

// ---------------------------------------------------------------------------
// Montgomery multiplication, R = 2^64, digit-serial REDC with 32-bit digits.
// For odd n < 2^64 and a, b < n returns a b R^-1 mod n in [0, n).
// The pre-subtraction value (a b + u n) / R is below 2n < 2^65, so its 65th
// bit is carried explicitly.  Ten 32-bit multiplies (all v_mad_u64_u32 /
// v_mul_lo_u32).
// ---------------------------------------------------------------------------
__device__ __forceinline__ u64 mont_mul(u64 a, u64 b, u64 n, u32 ninv) {
  const u32 a0 = lo32(a), a1 = hi32(a), b0 = lo32(b), b1 = hi32(b);
  const u32 n0 = lo32(n), n1 = hi32(n);
  // T = a b = th 2^64 + t1 2^32 + t0
  u64 p00 = (u64)a0 * b0;
  u64 p01 = mad32(a0, b1, hi32(p00));
  u64 p10 = mad32(a1, b0, lo32(p01));
  u64 th = mad32(a1, b1, hi32(p01)) + hi32(p10);
  u32 t0 = lo32(p00), t1 = lo32(p10);
  // digit 0: u = t0 (-n^-1) mod 2^32, T += u n, drop the zero digit
  u32 u = t0 * ninv;
  u64 q0 = mad32(u, n0, t0);                       // lo32(q0) == 0
  u64 q1 = mad32(u, n1, (u64)t1 + hi32(q0));       // <= 2^64 - 1
  u64 w = th + hi32(q1);
  u32 c = w < th;                                  // bit 2^128 of T + u n
  u32 d1 = lo32(q1);
  // digit 1
  u32 v = d1 * ninv;
  u64 r0 = mad32(v, n0, d1);                       // lo32(r0) == 0
  u64 r1 = mad32(v, n1, (u64)lo32(w) + hi32(r0));  // <= 2^64 - 1
  u64 top = (u64)hi32(w) + hi32(r1) + ((u64)c << 32);  // result = top 2^32 + lo32(r1) < 2n
  u64 res = (top << 32) | lo32(r1);
  bool c65 = (top >> 32) != 0;
  return (c65 || res >= n) ? res - n : res;
}

// Left-to-right square-and-multiply on plain (non-Montgomery) m: after the
// ladder x = m^E R^-(E-1) mod n; one more product with ce = R^E mod n gives
// m^E mod n.  L(E) + 1 products (Introduction: fewer than 2 log2 e).
template <u32 E>
__device__ __forceinline__ u64 mont_encrypt(u64 m, u64 n, u32 ninv, u64 ce) {
  static_assert(E >= 1, "exponent");
  u64 x = m;
  constexpr int top = 31 - __builtin_clz(E);
#pragma unroll
  for (int bit = top - 1; bit >= 0; --bit) {
    x = mont_mul(x, x, n, ninv);
    if ((E >> bit) & 1u) x = mont_mul(x, m, n, ninv);
  }
  return mont_mul(x, ce, n, ninv);
}

__device__ __forceinline__ u64 mont_encrypt_rt(u64 m, u64 n, u32 ninv, u64 ce, u32 e) {
  u64 x = m;
  int top = 31 - __builtin_clz(e);
  for (int bit = top - 1; bit >= 0; --bit) {
    x = mont_mul(x, x, n, ninv);
    if ((e >> bit) & 1u) x = mont_mul(x, m, n, ninv);
  }
  return mont_mul(x, ce, n, ninv);
}

// ---------------------------------------------------------------------------
// CRT with binary64 residues (Number Theory, eqs. CRTimplementation).
// A residue modulo a prime P < 2^32 is an integer-valued double in (-P, P).
// fmm(x, y): with |x|, |y| < P (or |x y| < 2^65 for Garner's product):
//   h = RN(x y), l = x y - h exactly (fma), qt = rint(h / P) within one of
//   round(x y / P), and h - qt P + l = x y - qt P is an integer of magnitude
//   below P that the fma and the add produce exactly.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double fmm(double x, double y, double P, double Pinv) {
  double h = x * y;
  double l = __fma_rn(x, y, -h);
  double qt = __builtin_rint(h * Pinv);
  return __fma_rn(-qt, P, h) + l;
}

// H K mod P up to a multiple of P, in (-P, P), for an integer-valued |H| < 2^35
// and a constant 0 <= K < P < 2^32 given split as K = hi + lo (hi a multiple of
// 2^17, lo < 2^17) with quo = RN(K RN(1/P)):
//   H hi and H lo are exact (below 2^50 and 2^52);
//   H quo is within 2^-16 of H K / P (|H K / P| < 2^35, three roundings of
//   relative size 2^-53), so qt = rint(H quo) is within 1/2 + 2^-16 of it and
//   r = H K - qt P lies in (-P, P);
//   fma(-qt, P, H hi) = r - H lo is an integer below 2^53 in magnitude (exact),
//   and the last fma adds H lo back exactly.
// Five operations, against six for the product split of fmm.
__device__ __forceinline__ double fold_split(double H, double P, double lo, double hi,
                                             double quo) {
  const double qt = __builtin_rint(H * quo);
  return __fma_rn(H, lo, __fma_rn(-qt, P, H * hi));
}

// m mod P from m = mh 2^32 + ml: (mh (2^32 mod P) + ml) reduced, in (-P, P).
__device__ __forceinline__ double residue(u64 m, double P, double Pinv, double lo, double hi,
                                          double quo) {
  const double t2 = fold_split((double)hi32(m), P, lo, hi, quo) + (double)lo32(m);  // |t2| < 2^33
  double qt = __builtin_rint(t2 * Pinv);
  return __fma_rn(-qt, P, t2);
}

// m mod P without the final reduction: an integer in (-P, P + 2^32).  Valid
// as the input of a squaring (|x|^2 < 2^66 keeps every fmm step exact: h < 2^67,
// |l| <= 2^14, |h - qt P| < P).
__device__ __forceinline__ double residue_lazy(u64 m, double P, double lo, double hi,
                                               double quo) {
  return fold_split((double)hi32(m), P, lo, hi, quo) + (double)lo32(m);
}

template <u32 E>
__device__ __forceinline__ double fp_pow(double x, double P, double Pinv) {
  double y = x;
  constexpr int top = 31 - __builtin_clz(E);
#pragma unroll
  for (int bit = top - 1; bit >= 0; --bit) {
    y = fmm(y, y, P, Pinv);
    if ((E >> bit) & 1u) y = fmm(y, x, P, Pinv);
  }
  return y;
}

__device__ __forceinline__ double fp_pow_rt(double x, double P, double Pinv, u32 e) {
  double y = x;
  int top = 31 - __builtin_clz(e);
  for (int bit = top - 1; bit >= 0; --bit) {
    y = fmm(y, y, P, Pinv);
    if ((e >> bit) & 1u) y = fmm(y, x, P, Pinv);
  }
  return y;
}

// x in (-P, P) (an integer) moved to [0, P): floor(x / P) is -1 or 0, and
// RN(x RN(1/P)) stays inside (-1, 1) on the right side of 0 for P < 2^52, so
// its floor decides; the fma then adds P exactly.  Arithmetic instead of a
// compare and select keeps the condition out of VCC.
__device__ __forceinline__ double to_unsigned_residue(double x, double P, double Pinv) {
  return __fma_rn(-__builtin_floor(x * Pinv), P, x);
}

// Garner's recombination c = ((c_p - c_q) q^-1 mod p) q + c_q.  Returns the
// integer c and RN(c) (one rounding of t q + c_q by the fma).  q^-1 mod p is
// given split (g_lo, g_hi, g_quo) as for fold_split; |d| < 2^33.
__device__ __forceinline__ u64 garner(double cp, double cq, double pd, double qd, double pinv,
                                      double qinv, double g_lo, double g_hi, double g_quo, u32 q,
                                      double& cd) {
  const double cqn = to_unsigned_residue(cq, qd, qinv);   // [0, q)
  const double d = cp - cqn;                              // exact, |d| < 2^33
  const double t = to_unsigned_residue(fold_split(d, pd, g_lo, g_hi, g_quo), pd, pinv);  // [0, p)
  cd = __fma_rn(t, qd, cqn);
  return mad32((u32)t, q, (u64)(u32)cqn);
}

// RN(c) for a 64-bit integer: both halves are exact doubles and the fma rounds
// hi 2^32 + lo once.
__device__ __forceinline__ double u64_to_f64_rn(u64 c) {
  return __fma_rn((double)hi32(c), 4294967296.0, (double)lo32(c));
}

// r = RN(RN(c) / RN(n)) with the guard against 1.0 (eq. CodeFloatingPointStep).
// With y = RN(1/nd) and its low part yl (y + yl = 1/nd to about 2^-105
// relative):
//   q0 = RN(cd y + RN(cd yl)) lies within half an ulp of cd/nd plus a relative
//   2^-103, so within one ulp;
//   hence cd - q0 nd is exactly representable and the fma returns it exactly,
//   and with y within half an ulp of 1/nd, q1 = RN(q0 + (cd - q0 nd) y) is the
//   correctly rounded cd/nd (Markstein's theorem, IBM J. Res. Dev. 1990).
// 0 <= cd <= nd: no underflow or overflow is possible.
__device__ __forceinline__ double ratio(double cd, double nd, double y, double yl) {
  const double q0 = __fma_rn(cd, y, cd * yl);
  const double r = __fma_rn(__fma_rn(-q0, nd, cd), y, q0);
  // r <= 1; the guard replaces exactly 1.0 by the largest double below it
  return __builtin_fmin(r, 0x1.fffffffffffffp-1);
}

}  // namespace rsaprng
