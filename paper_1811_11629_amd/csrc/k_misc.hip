// Small kernels (queue reset, statistics zero/finalise, test encryption) and
// the dispatch from a kernel shape to its tile-kernel family.
#include <algorithm>

#include "tiles.h"

namespace rsaprng {

static int hip_rc(hipError_t e) { return e == hipSuccess ? RSAPRNG_OK : RSAPRNG_E_HIP; }

// ---------------------------------------------------------------------------
// chain setup, sums, scan
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_chain_setup(LaunchArgs a) {
  const int lane = threadIdx.x & 63;
  const u32 c = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (c >= a.nchain) return;
  const Chain C = a.chain[c];
  for (u32 i = lane; i < C.ntiles; i += 64) a.tile_chain[C.first + i] = c;
  if (C.flags & kChainStartGiven) return;  // written by k_leadin_state
  const rsaprng_params P = a.inst[C.inst];
  const u64 n = P.n;
  u64 s_S, m_base;
  if (C.flags & kChainFromState) {
    const ChainState cs = a.state[C.slot];
    s_S = cs.s_at;
    m_base = cs.m_prev;
  } else {
    // a^S by the product over the set bits of S of a^(2^i), one bit per lane
    u64 f = ((C.S >> lane) & 1ull) ? a.pow2[lane] : 1ull;
#pragma unroll
    for (int m = 1; m < 64; m <<= 1) f = mulmod_q(f, __shfl_xor(f, m, 64));
    s_S = mulmod_q(P.s0, f);
    // S is a block start bB: m_bB = m0 + G_b, and the message "before" S is
    // m_bB - s_S so that adding the skip at S reproduces m_bB.
    const u64 G = mulmod_q(mulmod_q(P.s0, a.gc), f - 1);
    const u64 m_bs = addmod(P.m0, skip_mod_n(G, n), n);
    m_base = submod(m_bs, skip_mod_n(s_S, n), n);
  }
  if (lane == 0) {
    ChainStart cs;
    cs.s_S = s_S;
    cs.m_base = m_base;
    cs.rp = res_p(m_base, P);
    cs.rq = res_q(m_base, P);
    a.cstart[c] = cs;
  }
}

// One thread per lead-in chain (its tiles' chunk sums and prefixes already in
// agg and excl): the message at its last index is the prefix of its last chunk
// plus that chunk's sum, and the skip after it is the skip at its start times
// a^(T ntiles) (a lead-in chain lies inside one 2^20 block, so ntiles < 2^20 / T
// and the power is a table entry).  They become the start of the output chain
// named by its slot.
__global__ __launch_bounds__(256) void k_leadin_state(LaunchArgs a, ChainStart* out) {
  const u32 l = blockIdx.x * 256 + threadIdx.x;
  if (l >= a.nchain) return;
  const Chain L = a.chain[l];
  const rsaprng_params P = a.inst[L.inst];
  const u64 q = ((u64)(L.first + L.ntiles) << (a.tile_log2 - a.chunk_log2)) - 1;
  ChainStart cs;
  cs.m_base = addmod(a.excl[q], a.agg[q], P.n);
  cs.s_S = mulmod_q(a.cstart[l].s_S, a.at[L.ntiles]);
  cs.rp = res_p(cs.m_base, P);
  cs.rq = res_q(cs.m_base, P);
  out[L.slot] = cs;
}

// The sum of per (even) consecutive skips from s as lo + 2^64 hi.  Two
// reduced skips (each below 2^63) add without overflow, so the carry is taken
// once per pair; with LAZY the steps are lcg_lazy's and top their largest hi32
// (the sum is exact when it stays below kHiUnreduced).
template <bool LAZY>
__device__ __forceinline__ void lane_skip_sum(u64 s, int per, u64& lo, u32& hi, u32& top) {
  lo = 0;
  hi = 0;  // below per / 2: a 32-bit count, one add with the carry per pair
  for (int i = 0; i < per; i += 2) {
    if (i) s = walk_step<LAZY>(s, top);
    const u64 s1 = walk_step<LAZY>(s, top);
    const u64 pair = s + s1;
    const u64 t2 = lo + pair;
    hi += t2 < pair;
    lo = t2;
    s = s1;
  }
}

// One wave per tile: T/64 consecutive skips per lane; the sums of the tile's
// wave chunks (64 V indices each, 64/NW consecutive lanes here) mod n.
__global__ __launch_bounds__(256) void k_sums(LaunchArgs a) {
  const int lane = threadIdx.x & 63;
  const u32 t = uniform(blockIdx.x * 4 + (threadIdx.x >> 6));
  if (t >= a.ntiles) return;
  // wave-uniform records through the constant address space (scalar loads)
  const u32 c = cst(a.tile_chain)[t];
  const u32 first = cst(&a.chain[c].first)[0];
  const u32 inst = cst(&a.chain[c].inst)[0];
  const u64 n = cst(&a.inst[inst].n)[0];
  const u32 j = t - first;
  const u64 s_tile = mulmod_q(cst(&a.cstart[c].s_S)[0], cst(a.at)[j]);
  const u64 s0 = mulmod_q(s_tile, a.pl[lane]);
  const int per = 1 << (a.tile_log2 - 6);  // even: T >= 2048
  // exact integer sum of the lane's skips: lo + 2^64 hi, hi < per / 2 (skips <
  // 2^63); lazy steps first, the walk redone with reduced steps in a wave where
  // one of them may be unreduced
  u64 lo;
  u32 hi;
  u32 top = 0;
  lane_skip_sum<true>(s0, per, lo, hi, top);
  if (wave_any_unreduced(top)) lane_skip_sum<false>(s0, per, lo, hi, top);
  // reduce mod n: lo mod n (lo < 2^64 <= 4n), plus hi (2^64 mod n) by doubling
  u64 x = lo;
  x = x >= n ? x - n : x;
  x = x >= n ? x - n : x;
  x = x >= n ? x - n : x;
  u64 r64 = 0 - n;  // 2^64 - n < 3n
  r64 = r64 >= n ? r64 - n : r64;
  r64 = r64 >= n ? r64 - n : r64;
  u64 h = 0;
  for (int b = 31 - __builtin_clz(per); b >= 0; --b) {
    h = addmod(h, h, n);
    if ((hi >> b) & 1) h = addmod(h, r64, n);
  }
  x = addmod(x, h, n);
  const int nw_log2 = a.tile_log2 - a.chunk_log2;     // wave chunks per tile
  const int group = 64 >> nw_log2;                     // lanes per chunk
  // chunk sums as differences of the inclusive scan at the chunk boundaries
  const u64 incl = wave_scan_mod(x, n);
  const u64 before = __shfl(incl, (lane & ~(group - 1)) - 1 + (lane < group ? 64 : 0), 64);
  if ((lane & (group - 1)) == group - 1)
    a.agg[((u64)t << nw_log2) + (lane >> (6 - nw_log2))] =
        lane < group ? incl : submod(incl, before, n);
  if (lane == 0) a.s_tile[t] = s_tile;
}

// One wave per chain: excl[chunk] = message before the wave chunk.  A chain
// lies inside one block of 2^20 indices, so it has at most 2^20 / 512 = 2048
// chunks: lane l takes a run of up to kScanPer = 32 consecutive chunks, loads
// their sums at once, and after one wave scan of the run totals writes the
// run's prefixes in order.  A longer chain (none is planned) would take further
// rounds of 2048 chunks, carrying the message.
constexpr u32 kScanPer = 32;
__global__ __launch_bounds__(256) void k_scan(LaunchArgs a) {
  const int lane = threadIdx.x & 63;
  const u32 c = uniform(blockIdx.x * 4 + (threadIdx.x >> 6));
  if (c >= a.nchain) return;
  // wave-uniform records through the constant address space (scalar loads)
  const u32 ntiles = cst(&a.chain[c].ntiles)[0];
  const u32 first = cst(&a.chain[c].first)[0];
  const u64 n = cst(&a.inst[cst(&a.chain[c].inst)[0]].n)[0];
  const int nw_log2 = a.tile_log2 - a.chunk_log2;
  const u64 q_first = (u64)first << nw_log2;         // first chunk of the chain
  const u64 nq = (u64)ntiles << nw_log2;             // chunks of the chain
  const u32 inst = cst(&a.chain[c].inst)[0];
  u64 E = cst(&a.cstart[c].m_base)[0];
  for (u64 base = 0; base < nq; base += 64 * kScanPer) {
    const u64 left = nq - base;
    const u64 per = left >= 64 * kScanPer ? kScanPer : (left + 63) / 64;  // <= kScanPer
    const u64 q0 = base + (u64)lane * per;           // this lane's run [q0, q1)
    const u64 q1 = q0 + per < left + base ? q0 + per : left + base;
    u64 v[kScanPer];
#pragma unroll
    for (u32 j = 0; j < kScanPer; ++j) v[j] = q0 + j < q1 ? a.agg[q_first + q0 + j] : 0;
    u64 tot = 0;
#pragma unroll
    for (u32 j = 0; j < kScanPer; ++j) tot = addmod(tot, v[j], n);
    const u64 incl = wave_scan_mod(tot, n);
    u64 x = addmod(E, submod(incl, tot, n), n);      // message before the run
    if (a.excl_res) {
      // the residues of each message mod p and mod q (its run's sums are
      // already in registers, so the residue mod p can take their place)
      const rsaprng_params P = load_cst(a.inst + inst);
#pragma unroll
      for (u32 j = 0; j < kScanPer; ++j) {
        if (q0 + j < q1) {
          a.agg[q_first + q0 + j] = (u64)__double_as_longlong(res_p(x, P));
          a.excl[q_first + q0 + j] = (u64)__double_as_longlong(res_q(x, P));
        }
        x = addmod(x, v[j], n);
      }
    } else {
#pragma unroll
      for (u32 j = 0; j < kScanPer; ++j) {
        if (q0 + j < q1) a.excl[q_first + q0 + j] = x;
        x = addmod(x, v[j], n);
      }
    }
    E = addmod(E, lane_value(incl, 63), n);
  }
}

// ---------------------------------------------------------------------------
// small kernels
// ---------------------------------------------------------------------------
__global__ void k_begin(DevCtl* ctl) {
  ctl->counter = 0;
  u32 e = ctl->epoch + 1;
  ctl->epoch = e ? e : 1;
}

__global__ void k_stats_zero(rsaprng_stats* st, size_t nrec) {
  size_t words = nrec * (sizeof(rsaprng_stats) / 8);
  u64* w = reinterpret_cast<u64*>(st);
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < words;
       i += (size_t)gridDim.x * blockDim.x)
    w[i] = 0;
}

// 192-bit digits -> normalised limbs and the once-rounded double (ties to even).
__global__ void k_stats_finalize(rsaprng_stats* st, size_t nrec) {
  size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  if (i >= nrec) return;
  rsaprng_stats* s = st + i;
  u64 limb[3] = {0, 0, 0};
  u64 carry = 0;
  u32 dig[6];
  for (int j = 0; j < 6; ++j) {
    u64 v = s->acc32[j] + carry;   // acc32[j] < 2^63 by construction
    dig[j] = lo32(v);
    carry = v >> 32;
  }
  for (int j = 0; j < 3; ++j) limb[j] = ((u64)dig[2 * j + 1] << 32) | dig[2 * j];
  // canonical digits, so that the record does not depend on how the sum was split
  for (int j = 0; j < 6; ++j) s->acc32[j] = dig[j];
  s->sum_fx[0] = limb[0];
  s->sum_fx[1] = limb[1];
  s->sum_fx[2] = limb[2];
  // round the 192-bit integer to 53 bits, then scale by 2^-128
  int top = -1;
  for (int j = 2; j >= 0 && top < 0; --j)
    if (limb[j]) top = 64 * j + 63 - __builtin_clzll(limb[j]);
  double d = 0.0;
  if (top >= 0) {
    auto bit = [&](int b) -> u64 { return b < 0 ? 0 : (limb[b >> 6] >> (b & 63)) & 1ull; };
    int lsb = top - 52;  // position of the last kept bit
    u64 mant = 0;
    for (int b = top; b >= lsb && b >= 0; --b) mant = (mant << 1) | bit(b);
    if (lsb > 0) {
      u64 half = bit(lsb - 1);
      bool sticky = false;
      for (int b = lsb - 2; b >= 0; --b) sticky |= bit(b) != 0;
      if (half && (sticky || (mant & 1))) ++mant;
      d = ldexp((double)mant, lsb - 128);
    } else {
      d = ldexp((double)mant, -128);
    }
  }
  s->sum = d;
}

// Position-dependent fingerprint of a buffer of 64-bit words (order-independent
// sum of mixed (index, value) pairs), used to check that kernel configurations
// produce identical bytes without copying outputs to the host.
__device__ __forceinline__ u64 mix64(u64 z) {
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

__global__ void k_checksum(const u64* p, u64 n, u64* out) {
  u64 acc = 0;
  for (u64 i = blockIdx.x * (u64)blockDim.x + threadIdx.x; i < n; i += (u64)gridDim.x * blockDim.x)
    acc += mix64(p[i] ^ mix64(i + 0x9e3779b97f4a7c15ull));
  for (int m = 1; m < 64; m <<= 1) acc += __shfl_xor(acc, m, 64);
  if ((threadIdx.x & 63) == 0) atomicAdd((unsigned long long*)out, (unsigned long long)acc);
}

__global__ void k_zero1(u64* p) { *p = 0; }

int launch_checksum(const uint64_t* p, uint64_t n, uint64_t* out_dev, void* stream) {
  hipLaunchKernelGGL(k_zero1, dim3(1), dim3(1), 0, (hipStream_t)stream, out_dev);
  if (n) hipLaunchKernelGGL(k_checksum, dim3(2048), dim3(256), 0, (hipStream_t)stream, p, n, out_dev);
  return hip_rc(hipGetLastError());
}

__global__ void k_fill(u64* p, u64 n, u64 v) {
  for (u64 i = blockIdx.x * (u64)blockDim.x + threadIdx.x; i < n; i += (u64)gridDim.x * blockDim.x)
    p[i] = v;
}

int launch_fill(uint64_t* p, uint64_t n, uint64_t v, void* stream) {
  if (n) hipLaunchKernelGGL(k_fill, dim3(2048), dim3(256), 0, (hipStream_t)stream, p, n, v);
  return hip_rc(hipGetLastError());
}

template <int VAR>
__global__ void k_debug_encrypt(rsaprng_params P, const u64* m, u64* c, double* r, u64 count) {
  u64 i = blockIdx.x * (u64)blockDim.x + threadIdx.x;
  if (i >= count) return;
  double cd;
  u64 v = encrypt<VAR, 0>(m[i], P, cd);
  if (c) c[i] = v;
  if (r) r[i] = ratio_of(cd, P);
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

int launch_begin(DevCtl* ctl, void* stream) {
  hipLaunchKernelGGL(k_begin, dim3(1), dim3(1), 0, (hipStream_t)stream, ctl);
  return hip_rc(hipGetLastError());
}

int launch_chain_setup(const LaunchArgs& a, void* stream) {
  if (!a.nchain) return RSAPRNG_OK;
  hipLaunchKernelGGL(k_chain_setup, dim3((a.nchain + 3) / 4), dim3(256), 0, (hipStream_t)stream, a);
  return hip_rc(hipGetLastError());
}

int launch_leadin_state(const LaunchArgs& a, ChainStart* out, void* stream) {
  if (!a.nchain) return RSAPRNG_OK;
  hipLaunchKernelGGL(k_leadin_state, dim3((a.nchain + 255) / 256), dim3(256), 0,
                     (hipStream_t)stream, a, out);
  return hip_rc(hipGetLastError());
}

int launch_sums(const LaunchArgs& a, void* stream) {
  if (!a.ntiles) return RSAPRNG_OK;
  hipLaunchKernelGGL(k_sums, dim3((a.ntiles + 3) / 4), dim3(256), 0, (hipStream_t)stream, a);
  return hip_rc(hipGetLastError());
}

int launch_scan(const LaunchArgs& a, void* stream) {
  if (!a.nchain) return RSAPRNG_OK;
  hipLaunchKernelGGL(k_scan, dim3((a.nchain + 3) / 4), dim3(256), 0, (hipStream_t)stream, a);
  return hip_rc(hipGetLastError());
}

int launch_mont_gen(const KernelShape&, const LaunchArgs&, void*, int*);
int launch_crt_gen(const KernelShape&, const LaunchArgs&, void*, int*);
int launch_mont_con(const KernelShape&, const LaunchArgs&, void*, int*);
int launch_crt_con(const KernelShape&, const LaunchArgs&, void*, int*);
int launch_crt_bat(const KernelShape&, const LaunchArgs&, void*, int*);

static int dispatch(const KernelShape& s, const LaunchArgs* a, void* stream, int* occ) {
  static const LaunchArgs dummy{};
  const LaunchArgs& aa = a ? *a : dummy;
  if (s.variant == kVariantMont && s.mode == kModeGenerate) return launch_mont_gen(s, aa, stream, occ);
  if (s.variant == kVariantCrt && s.mode == kModeGenerate) return launch_crt_gen(s, aa, stream, occ);
  if (s.variant == kVariantMont && s.mode == kModeConsume) return launch_mont_con(s, aa, stream, occ);
  if (s.variant == kVariantCrt && s.mode == kModeConsume) return launch_crt_con(s, aa, stream, occ);
  if (s.variant == kVariantCrt && s.mode == kModeBattery) return launch_crt_bat(s, aa, stream, occ);
  return RSAPRNG_E_ARG;
}

int launch_tiles(const KernelShape& s, const LaunchArgs& a, void* stream) {
  return dispatch(s, &a, stream, nullptr);
}

int kernel_max_grid(const KernelShape& s, int* wg_per_cu) { return dispatch(s, nullptr, nullptr, wg_per_cu); }

// Clears a battery record word by word (a kernel, so that graph capture
// records no memset node) and sets its output count (the first word).
__global__ __launch_bounds__(256) void k_battery_zero(uint64_t* w, size_t nwords, uint64_t outputs) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < nwords;
       i += (size_t)gridDim.x * blockDim.x)
    w[i] = i == 0 ? outputs : 0;
}

int launch_battery_zero(rsaprng_battery* rec, uint64_t outputs, void* stream) {
  const size_t nwords = sizeof(rsaprng_battery) / 8;
  hipLaunchKernelGGL(k_battery_zero, dim3(2048), dim3(256), 0, (hipStream_t)stream,
                     reinterpret_cast<uint64_t*>(rec), nwords, outputs);
  return hip_rc(hipGetLastError());
}

int launch_stats_zero(rsaprng_stats* st, size_t nrec, void* stream) {
  size_t words = nrec * (sizeof(rsaprng_stats) / 8);
  int grid = (int)std::min<size_t>((words + 255) / 256, 4096);
  if (grid < 1) grid = 1;
  hipLaunchKernelGGL(k_stats_zero, dim3(grid), dim3(256), 0, (hipStream_t)stream, st, nrec);
  return hip_rc(hipGetLastError());
}

int launch_stats_finalize(rsaprng_stats* st, size_t nrec, void* stream) {
  int grid = (int)((nrec + 127) / 128);
  if (grid < 1) grid = 1;
  hipLaunchKernelGGL(k_stats_finalize, dim3(grid), dim3(128), 0, (hipStream_t)stream, st, nrec);
  return hip_rc(hipGetLastError());
}

int launch_debug_encrypt(const rsaprng_params& prm, int variant, const uint64_t* m, uint64_t* c,
                         double* r, uint64_t count, void* stream) {
  if (count == 0) return RSAPRNG_OK;
  u64 grid = (count + 255) / 256;
  if (grid > 0x7fffffffull) return RSAPRNG_E_RANGE;
  if (variant == kVariantMont)
    hipLaunchKernelGGL(k_debug_encrypt<kVariantMont>, dim3((u32)grid), dim3(256), 0,
                       (hipStream_t)stream, prm, m, c, r, count);
  else
    hipLaunchKernelGGL(k_debug_encrypt<kVariantCrt>, dim3((u32)grid), dim3(256), 0,
                       (hipStream_t)stream, prm, m, c, r, count);
  return hip_rc(hipGetLastError());
}

}  // namespace rsaprng
