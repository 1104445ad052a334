// gfx950 kernels of the RSA-exponentiation generator.
//
// One work-group processes one tile of T = WG * V consecutive indices of one
// request (V per lane).  Per tile:
//   1. jump   : s at the tile start, s0 a^K mod Q, by a product tree of the
//               table a^(2^i) across the 64 lanes of wave 0 (eq. pseudoskip for
//               the skips); at a block start also the block seed
//               G_b = s0 a (a^{bB} - 1) / (a - 1) mod Q;
//   2. walk   : each lane steps its V skips (eq. congruentialgenerator1) and
//               keeps their running sums mod n in registers;
//   3. scan   : wave scan + LDS across waves gives each lane's offset and the
//               tile aggregate; the message before the tile comes from a
//               decoupled look-back over the preceding tiles of the same block
//               (tagged 64-bit words, relaxed agent-scope atomics, bounded wait);
//   4. encrypt: c = m^e mod n per element (Montgomery-64 or CRT/binary64),
//               r = RN(c)/RN(n) with the 1.0 guard;
//   5. store  : c, r to HBM (generate) or fold into exact statistics (consume).
// Tile ids come from an atomic counter, so a tile only ever waits on tiles that
// were claimed before it by resident work-groups, and every wait is bounded.
#pragma once
#include "common.h"
#include "devmath.h"

namespace rsaprng {

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

__device__ __forceinline__ u64 wave_sum_mod(u64 v, u64 n) {
#pragma unroll
  for (int m = 1; m < 64; m <<= 1) v = addmod(v, __shfl_xor(v, m, 64), n);
  return v;
}

// Exclusive prefix (mod n) of tile t: the inclusive value of the nearest
// predecessor that has one plus the aggregates in between.  Executed by one
// full wave; the chain's first tile always publishes an inclusive value.
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
      __builtin_amdgcn_s_sleep(2);
    }
    u64 imask = __ballot(valid && hasI);
    int stop = imask ? __ffsll((unsigned long long)imask) - 1 : 64;
    u64 contrib = 0;
    if (valid) contrib = lane < stop ? va : (lane == stop ? vi : 0);
    acc = addmod(acc, wave_sum_mod(contrib, n), n);
    if (imask) return acc;
    pos -= 64;
  }
}

// ---------------------------------------------------------------------------
// encryption of one message
// ---------------------------------------------------------------------------
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
    double mp = residue(m, P.pd, P.pinv, P.kp);
    double mq = residue(m, P.qd, P.qinv, P.kq);
    double cp, cq;
    if constexpr (E != 0) {
      cp = fp_pow<E>(mp, P.pd, P.pinv);
      cq = fp_pow<E>(mq, P.qd, P.qinv);
    } else {
      cp = fp_pow_rt(mp, P.pd, P.pinv, P.e);
      cq = fp_pow_rt(mq, P.qd, P.qinv, P.e);
    }
    return garner(cp, cq, P.pd, P.qd, P.pinv, P.qinvp, P.q, cd);
  }
}

// r * 2^128 as a 128-bit integer (r = 0 or 2^-64 <= r < 1, so the shift is in [12, 75]).
__device__ __forceinline__ void fixed128(double r, u64& lo, u64& hi) {
  u64 bits = (u64)__double_as_longlong(r);
  int ex = (int)(bits >> 52);
  u64 mant = (bits & 0xfffffffffffffull) | (1ull << 52);
  int sh = ex - 947;
  if (ex == 0) {
    lo = 0;
    hi = 0;
  } else if (sh < 64) {
    lo = mant << sh;
    hi = mant >> (64 - sh);
  } else {
    lo = 0;
    hi = mant << (sh - 64);
  }
}

template <int V>
__device__ __forceinline__ void store_lane(u64* oc, double* orr, const u64 (&c)[V],
                                           const double (&r)[V]) {
  if (oc) {
    if (((uintptr_t)oc & 15) == 0) {
#pragma unroll
      for (int i = 0; i < V; i += 2)
        *reinterpret_cast<ulonglong2*>(oc + i) = make_ulonglong2(c[i], c[i + 1]);
    } else {
#pragma unroll
      for (int i = 0; i < V; ++i) oc[i] = c[i];
    }
  }
  if (orr) {
    if (((uintptr_t)orr & 15) == 0) {
#pragma unroll
      for (int i = 0; i < V; i += 2)
        *reinterpret_cast<double2*>(orr + i) = make_double2(r[i], r[i + 1]);
    } else {
#pragma unroll
      for (int i = 0; i < V; ++i) orr[i] = r[i];
    }
  }
}

template <int WG, int MODE>
struct TileShared {
  u32 tile;
  u64 s_tile;
  u64 pre;
  u64 wave_tot[WG / 64];
  u64 red[MODE == kModeConsume ? (WG / 64) * 6 : 1];
  u32 hist[MODE == kModeConsume ? 1024 : 1];
};

// Encryption, output and end-state phase of one tile for exponent E (0 = any).
template <int WG, int V, int VAR, int MODE, u32 E>
__device__ __forceinline__ void tile_outputs(const LaunchArgs& a, TileShared<WG, MODE>& sh,
                                             const Req& R, const rsaprng_params& P, u64 pre,
                                             const u64 (&X)[V], u64 laneStart) {
  const u64 n = P.n;
  const u64 last = R.k0 + (R.count - 1);
  const bool full = laneStart >= R.k0 && laneStart + (V - 1) <= last;
  if constexpr (MODE == kModeGenerate) {
    u64 c[V];
    double r[V];
#pragma unroll
    for (int i = 0; i < V; ++i) {
      double cd;
      c[i] = encrypt<VAR, E>(addmod(pre, X[i], n), P, cd);
      r[i] = ratio(cd, P.nd);
    }
    if (full) {
      u64 off = R.out_off + (laneStart - R.k0);
      store_lane<V>(a.out_c ? a.out_c + off : nullptr, a.out_r ? a.out_r + off : nullptr, c, r);
    } else {
#pragma unroll
      for (int i = 0; i < V; ++i) {
        u64 k = laneStart + i;
        if (k >= R.k0 && k <= last) {
          u64 off = R.out_off + (k - R.k0);
          if (a.out_c) a.out_c[off] = c[i];
          if (a.out_r) a.out_r[off] = r[i];
        }
      }
    }
  } else {
    u64 c0 = 0, c1 = 0, c2 = 0, c3 = 0, lt = 0, cnt = 0;
#pragma unroll
    for (int i = 0; i < V; ++i) {
      u64 k = laneStart + i;
      double cd;
      (void)encrypt<VAR, E>(addmod(pre, X[i], n), P, cd);
      double r = ratio(cd, P.nd);
      if (full || (k >= R.k0 && k <= last)) {
        u64 lo, hi;
        fixed128(r, lo, hi);
        c0 += lo32(lo);
        c1 += hi32(lo);
        c2 += lo32(hi);
        c3 += hi32(hi);
        lt += r < 0.5;
        cnt += 1;
        atomicAdd(&sh.hist[(int)(r * 1024.0)], 1u);
      }
    }
    // wave reductions (each chunk sum stays below 2^42)
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int m = 1; m < 64; m <<= 1) {
      c0 += __shfl_xor(c0, m, 64);
      c1 += __shfl_xor(c1, m, 64);
      c2 += __shfl_xor(c2, m, 64);
      c3 += __shfl_xor(c3, m, 64);
      lt += __shfl_xor(lt, m, 64);
      cnt += __shfl_xor(cnt, m, 64);
    }
    if (lane == 0) {
      u64* rd = sh.red + wave * 6;
      rd[0] = c0; rd[1] = c1; rd[2] = c2; rd[3] = c3; rd[4] = lt; rd[5] = cnt;
    }
    __syncthreads();
    rsaprng_stats* st = a.stats + R.slot;
    if (threadIdx.x == 0) {
      u64 s[4] = {0, 0, 0, 0}, tl = 0, tc = 0;
      for (int w = 0; w < WG / 64; ++w) {
        for (int j = 0; j < 4; ++j) s[j] += sh.red[w * 6 + j];
        tl += sh.red[w * 6 + 4];
        tc += sh.red[w * 6 + 5];
      }
      // carry-normalise into 32-bit digits so each atomic adds < 2^32
      u64 carry = 0;
      u32 dig[6];
      for (int j = 0; j < 4; ++j) {
        u64 v = s[j] + carry;
        dig[j] = lo32(v);
        carry = v >> 32;
      }
      dig[4] = lo32(carry);
      dig[5] = hi32(carry);
      for (int j = 0; j < 6; ++j)
        if (dig[j]) atomicAdd((unsigned long long*)&st->acc32[j], (unsigned long long)dig[j]);
      if (tl) atomicAdd((unsigned long long*)&st->lt_half, (unsigned long long)tl);
      if (tc) atomicAdd((unsigned long long*)&st->count, (unsigned long long)tc);
    }
    for (int b = threadIdx.x; b < 1024; b += WG) {
      u32 h = sh.hist[b];
      if (h) {
        atomicAdd((unsigned long long*)&st->hist[b], (unsigned long long)h);
        sh.hist[b] = 0;
      }
    }
  }
}

template <int WG, int V, int VAR, int MODE>
__global__ __launch_bounds__(WG) void k_tiles(LaunchArgs a) {
  constexpr int T = WG * V;
  constexpr int NW = WG / 64;
  __shared__ TileShared<WG, MODE> sh;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const u32 tag = a.ctl->epoch;

  if constexpr (MODE == kModeConsume) {
    for (int b = threadIdx.x; b < 1024; b += WG) sh.hist[b] = 0;
  }

  for (;;) {
    if (threadIdx.x == 0) sh.tile = atomicAdd(&a.ctl->counter, 1u);
    __syncthreads();
    const u32 t = __builtin_amdgcn_readfirstlane(sh.tile);
    if (t >= a.ntiles) break;

    // request owning tile t: the last one with tile_begin <= t
    u32 lo = 0, hi = a.nreq - 1;
    while (lo < hi) {
      u32 mid = (lo + hi + 1) >> 1;
      if (a.req[mid].tile_begin <= t) lo = mid; else hi = mid - 1;
    }
    const Req R = a.req[lo];
    const rsaprng_params P = a.inst[R.inst];
    const u64 n = P.n;
    const u32 j = t - R.tile_begin;
    const u64 tileStart = R.S + (u64)j * T;
    const u64 bs = tileStart & ~(kBlock - 1);
    const bool cont = (R.flags & kReqContinue) != 0;
    const bool from_state = cont && bs <= R.S;        // tile lies in the chain started from state
    const bool chain_start = from_state ? (j == 0) : (tileStart == bs);
    const u64 chainS = from_state ? R.S : bs;
    const u32 first = R.tile_begin + (u32)((chainS - R.S) / T);

    // 1. jump (wave 0)
    u64 mbase = 0;
    if (wave == 0) {
      u64 base, K;
      if (from_state) {
        const ChainState cs = a.state[R.slot];
        base = cs.s_at;
        K = tileStart - R.S;
        mbase = cs.m_prev;
      } else {
        base = P.s0;
        K = tileStart;
      }
      u64 f = ((K >> lane) & 1ull) ? a.pow2[lane] : 1ull;
#pragma unroll
      for (int m = 1; m < 64; m <<= 1) f = mulmod_q(f, __shfl_xor(f, m, 64));
      const u64 s_tile = mulmod_q(base, f);
      if (chain_start && !from_state) {
        // block seed: m_bs = m0 + G_b, G_b = s0 a (a^bs - 1)/(a - 1) mod Q; mbase = m_bs - s_bs
        u64 G = mulmod_q(mulmod_q(P.s0, a.gc), f - 1);
        u64 mbs = addmod(P.m0, skip_mod_n(G, n), n);
        u64 sn = skip_mod_n(s_tile, n);
        mbase = addmod(mbs, sn == 0 ? 0 : n - sn, n);
      } else if (chain_start && from_state) {
        // mbase already m_{S-1}
      }
      if (lane == 0) sh.s_tile = s_tile;
    }
    __syncthreads();

    // 2. walk
    const u64 laneStart = tileStart + (u64)threadIdx.x * V;
    u64 X[V];
    u64 s = mulmod_q(sh.s_tile, a.powv[threadIdx.x]);
    u64 s_first = s;
    u64 x = 0;
#pragma unroll
    for (int i = 0; i < V; ++i) {
      if (i) s = lcg_next(s);
      x = addmod(x, skip_mod_n(s, n), n);
      X[i] = x;
    }

    // 3. scan
    u64 incl = x;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      u64 y = __shfl_up(incl, d, 64);
      if (lane >= d) incl = addmod(incl, y, n);
    }
    u64 lane_excl = __shfl_up(incl, 1, 64);
    if (lane == 0) lane_excl = 0;
    if (lane == 63) sh.wave_tot[wave] = incl;
    __syncthreads();
    u64 wave_off = 0, agg = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w) {
      u64 v = sh.wave_tot[w];
      if (w < wave) wave_off = addmod(wave_off, v, n);
      agg = addmod(agg, v, n);
    }
    if (wave == 0) {
      u64 E;
      if (chain_start) {
        E = mbase;
      } else {
        if (lane == 0) publish(a.lb + 4ull * t, tag, agg);
        E = look_back(a, t, first, tag, n, lane);
      }
      if (lane == 0) {
        publish(a.lb + 4ull * t + 2, tag, addmod(E, agg, n));
        sh.pre = E;
      }
    }
    __syncthreads();
    const u64 pre = addmod(addmod(sh.pre, wave_off, n), lane_excl, n);

    // 4-5. outputs (only tiles that reach the requested range)
    if (tileStart + (T - 1) >= R.k0) {
      switch (P.e) {
        case 1: tile_outputs<WG, V, VAR, MODE, 1>(a, sh, R, P, pre, X, laneStart); break;
        case 3: tile_outputs<WG, V, VAR, MODE, 3>(a, sh, R, P, pre, X, laneStart); break;
        case 5: tile_outputs<WG, V, VAR, MODE, 5>(a, sh, R, P, pre, X, laneStart); break;
        case 7: tile_outputs<WG, V, VAR, MODE, 7>(a, sh, R, P, pre, X, laneStart); break;
        case 17: tile_outputs<WG, V, VAR, MODE, 17>(a, sh, R, P, pre, X, laneStart); break;
        case 257: tile_outputs<WG, V, VAR, MODE, 257>(a, sh, R, P, pre, X, laneStart); break;
        case 65537: tile_outputs<WG, V, VAR, MODE, 65537>(a, sh, R, P, pre, X, laneStart); break;
        default: tile_outputs<WG, V, VAR, MODE, 0>(a, sh, R, P, pre, X, laneStart); break;
      }
    }
    // chain-end state (served continuation): the lane holding the last index
    const u64 last = R.k0 + (R.count - 1);
    if ((R.flags & kReqWriteEnd) && laneStart <= last && last - laneStart < (u64)V) {
      u64 m_end = 0;
      u64 ss = s_first;
#pragma unroll
      for (int i = 0; i < V; ++i) {
        if (laneStart + i == last) m_end = addmod(pre, X[i], n);
        if (laneStart + i < last) ss = lcg_next(ss);
      }
      ChainState cs;
      cs.m_prev = m_end;
      cs.s_at = lcg_next(ss);
      a.state[R.slot] = cs;
    }
  }
}

template <int WG, int V, int VAR, int MODE>
static int launch_one(const LaunchArgs& a, int grid, void* stream) {
  hipLaunchKernelGGL((k_tiles<WG, V, VAR, MODE>), dim3(grid), dim3(WG), 0, (hipStream_t)stream, a);
  return hipGetLastError() == hipSuccess ? RSAPRNG_OK : RSAPRNG_E_HIP;
}

template <int WG, int V, int VAR, int MODE>
static int occupancy_of() {
  int blocks = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_tiles<WG, V, VAR, MODE>, WG, 0) !=
      hipSuccess)
    return 1;
  return blocks > 0 ? blocks : 1;
}

// Launcher and occupancy query for every tile shape of one (variant, mode).
template <int VAR, int MODE>
int launch_family(const KernelShape& s, const LaunchArgs& a, void* stream, int* occ) {
  if (s.wg == 256 && s.v == 16) {
    if (occ) { *occ = occupancy_of<256, 16, VAR, MODE>(); return RSAPRNG_OK; }
    return launch_one<256, 16, VAR, MODE>(a, s.grid, stream);
  }
  if (s.wg == 256 && s.v == 8) {
    if (occ) { *occ = occupancy_of<256, 8, VAR, MODE>(); return RSAPRNG_OK; }
    return launch_one<256, 8, VAR, MODE>(a, s.grid, stream);
  }
  if (s.wg == 128 && s.v == 16) {
    if (occ) { *occ = occupancy_of<128, 16, VAR, MODE>(); return RSAPRNG_OK; }
    return launch_one<128, 16, VAR, MODE>(a, s.grid, stream);
  }
  return RSAPRNG_E_ARG;
}

}  // namespace rsaprng
