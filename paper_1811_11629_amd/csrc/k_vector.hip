// Vector mode (Parallelization section, eq. vectorize and the stream
// splitting after it): M_v substreams of one instance advanced together.
// Substream g has the skip seed s0 a^(g J) mod Q with J = floor((Q-1)/M_v) and
// the instance's message seed m0, and is otherwise the instance's sequence
// (same n, e, block re-seeding).  Vector call t = 1, 2, ... returns element g
// = the output of substream g after t updates, i.e. its index k = t; the
// flattened output f = (t - 1) M_v + g.
//
// Layout of the work: one lane per (substream, segment of W = 2^w consecutive
// indices), substreams varying fastest, so that at every step the lanes of a
// wave store consecutive outputs of one vector call (512 contiguous bytes per
// store instruction when M_v >= 64).  The message before each segment comes
// from a scan along the substream:
//   k_vjump   s0 a^(g J) per substream and a^(sigma W) per segment;
//   k_vsums   the sum of each segment's skips mod n;
//   k_vscan1  exclusive prefixes inside groups of G = min(64, 2^20/W)
//             consecutive segments, and the group totals;
//   k_vscan2  per (substream, block): the block seed m_bB = m0 + G_b and the
//             exclusive prefix over the block's groups;
//   k_vgen    each lane walks its segment: skip step, message update,
//             encryption, r = c/n, stores.
// W <= 2^19, so a block holds at least two segments; segments never cross a
// block and the domain of a launch starts at a block start, so every prefix
// starts from a block seed.
#include "tiles.h"

namespace rsaprng {

namespace {

// a^x mod Q for any 64-bit x, from the table a^(2^i) (a^(Q-1) = 1, so this is
// also a^(x mod (Q-1))).
__device__ __forceinline__ u64 pow_a(const u64* pow2, u64 x) {
  u64 f = 1;
  for (int i = 0; i < 64; ++i)
    if ((x >> i) & 1ull) f = mulmod_q(f, pow2[i]);
  return f;
}

// lo + 2^64 hi mod n, hi < 2^32 (n > 2^62: lo < 4n and 2^64 mod n < 3n).
__device__ __forceinline__ u64 wide_mod_n(u64 lo, u32 hi, u64 n) {
  u64 x = lo;
  x = x >= n ? x - n : x;
  x = x >= n ? x - n : x;
  x = x >= n ? x - n : x;
  u64 r64 = 0 - n;
  r64 = r64 >= n ? r64 - n : r64;
  r64 = r64 >= n ? r64 - n : r64;
  u64 h = 0;
  for (int b = hi ? 31 - __builtin_clz(hi) : -1; b >= 0; --b) {
    h = addmod(h, h, n);
    if ((hi >> b) & 1u) h = addmod(h, r64, n);
  }
  return addmod(x, h, n);
}

__device__ __forceinline__ u32 gid() { return blockIdx.x * 256u + threadIdx.x; }

__global__ __launch_bounds__(256) void k_vjump(VecArgs a) {
  const u32 L = gid();
  if (L < a.ng) {
    u64 g = a.g_lo + L;
    g = g >= a.mv ? g - a.mv : g;
    a.va[L] = mulmod_q(a.P.s0, pow_a(a.pow2, g * a.J));  // g J < Q - 1
  } else if (L < a.ng + a.nseg) {
    const u32 i = L - a.ng;
    a.vb[i] = pow_a(a.pow2, (a.sig_a + i) << a.w);
  }
}

// Sum of the W skips of segment i of substream lane j, mod n.
__global__ __launch_bounds__(256) void k_vsums(VecArgs a) {
  const u32 L = gid();
  if (L >= a.nseg * a.ng) return;
  const u32 i = L / a.ng, j = L - i * a.ng;
  u64 s = mulmod_q(a.va[j], a.vb[i]);
  u64 lo = s;
  u32 hi = 0;
  const u32 W = 1u << a.w;
  for (u32 x = 1; x < W; ++x) {
    s = lcg_next(s);
    const u64 t = lo + s;
    hi += t < lo;
    lo = t;
  }
  a.vagg[L] = wide_mod_n(lo, hi, a.P.n);
}

// Exclusive prefixes inside each group of G segments (in place) and the group
// totals.
__global__ __launch_bounds__(256) void k_vscan1(VecArgs a) {
  const u32 L = gid();
  if (L >= a.ngrp * a.ng) return;
  const u32 grp = L / a.ng, j = L - grp * a.ng;
  const u64 n = a.P.n;
  const u32 i0 = grp << a.glog2;
  const u32 i1 = min(i0 + (1u << a.glog2), a.nseg);
  u64 acc = 0;
  for (u32 i = i0; i < i1; ++i) {
    const u64 v = a.vagg[(u64)i * a.ng + j];
    a.vagg[(u64)i * a.ng + j] = acc;
    acc = addmod(acc, v, n);
  }
  a.vgrp[L] = acc;
}

// Per (block, substream lane): the message before the block start from the
// block seed, then the message before each group of the block.
__global__ __launch_bounds__(256) void k_vscan2(VecArgs a) {
  const u32 L = gid();
  if (L >= a.nblk * a.ng) return;
  const u32 b = L / a.ng, j = L - b * a.ng;
  const u64 n = a.P.n;
  const u32 spb_log2 = kBlockLog2 - a.w;            // segments per block
  const u64 aB = a.vb[(u64)b << spb_log2];          // a^(bB), block b of the domain
  const u64 s0g = a.va[j];
  const u64 sB = mulmod_q(s0g, aB);                 // the skip at the block start
  const u64 G = mulmod_q(mulmod_q(s0g, a.gc), aB - 1);
  const u64 m_bs = addmod(a.P.m0, skip_mod_n(G, n), n);
  u64 acc = submod(m_bs, skip_mod_n(sB, n), n);    // message "before" bB
  const u32 gpb_log2 = spb_log2 - a.glog2;          // groups per block
  const u32 g0 = b << gpb_log2;
  const u32 g1 = min(g0 + (1u << gpb_log2), a.ngrp);
  for (u32 grp = g0; grp < g1; ++grp) {
    const u64 idx = (u64)grp * a.ng + j;
    const u64 v = a.vgrp[idx];
    a.vgrp[idx] = acc;
    acc = addmod(acc, v, n);
  }
}

template <int VAR, u32 E>
__device__ __forceinline__ void vgen_lane(const VecArgs& a, const rsaprng_params& P) {
  const u32 L = gid();
  if (L >= a.noseg * a.ng) return;
  const u32 io = L / a.ng, j = L - io * a.ng;
  const u32 i = a.osig + io;
  const u64 n = P.n;
  u64 g = a.g_lo + j;
  g = g >= a.mv ? g - a.mv : g;
  u64 m = addmod(a.vgrp[(u64)(i >> a.glog2) * a.ng + j], a.vagg[(u64)i * a.ng + j], n);
  u64 s = mulmod_q(a.va[j], a.vb[i]);
  const u64 k0 = (a.sig_a + i) << a.w;
  // indices of this segment up to the last vector call of the launch; those
  // before the first call only advance the message
  const u64 kend = a.t_hi - k0 + 1;
  const u32 W = 1u << a.w;
  const u32 xend = kend < W ? (u32)kend : W;
  const u32 xout = a.t_lo > k0 ? (u32)(a.t_lo - k0) : 0u;  // <= xend
  u32 x = 0;
  for (; x < xout; ++x) {
    if (x) s = lcg_next(s);
    m = addmod(m, skip_mod_n(s, n), n);
  }
  // output offset f - f0 = (k - t_lo) M_v + g - g_lo, negative only in the
  // first call for g < g_lo; it advances by M_v per index
  long long o = (long long)((k0 + x - a.t_lo) * a.mv + g) - (long long)a.g_lo;
  const long long cnt = (long long)a.count;
  const long long step = (long long)a.mv;
  for (; x < xend; ++x, o += step) {
    if (x) s = lcg_next(s);
    m = addmod(m, skip_mod_n(s, n), n);
    if (o < 0 || o >= cnt) continue;
    double cd;
    const u64 c = encrypt<VAR, E>(m, P, cd);
    if (a.out_c) a.out_c[o] = c;
    if (a.out_r) a.out_r[o] = ratio_of(cd, P);
  }
}

template <int VAR>
__global__ __launch_bounds__(256) void k_vgen(VecArgs a) {
  const rsaprng_params& P = a.P;
  switch (P.e) {
    case 1: vgen_lane<VAR, 1>(a, P); break;
    case 3: vgen_lane<VAR, 3>(a, P); break;
    case 5: vgen_lane<VAR, 5>(a, P); break;
    case 7: vgen_lane<VAR, 7>(a, P); break;
    case 17: vgen_lane<VAR, 17>(a, P); break;
    case 257: vgen_lane<VAR, 257>(a, P); break;
    case 65537: vgen_lane<VAR, 65537>(a, P); break;
    default: vgen_lane<VAR, 0>(a, P); break;
  }
}

inline dim3 grid_for_lanes(u64 lanes) { return dim3((u32)((lanes + 255) / 256)); }

}  // namespace

int launch_vector(const VecArgs& a, int variant, void* stream) {
  hipStream_t st = (hipStream_t)stream;
  hipLaunchKernelGGL(k_vjump, grid_for_lanes((u64)a.ng + a.nseg), dim3(256), 0, st, a);
  hipLaunchKernelGGL(k_vsums, grid_for_lanes((u64)a.nseg * a.ng), dim3(256), 0, st, a);
  hipLaunchKernelGGL(k_vscan1, grid_for_lanes((u64)a.ngrp * a.ng), dim3(256), 0, st, a);
  hipLaunchKernelGGL(k_vscan2, grid_for_lanes((u64)a.nblk * a.ng), dim3(256), 0, st, a);
  const dim3 gg = grid_for_lanes((u64)a.noseg * a.ng);
  if (variant == kVariantMont)
    hipLaunchKernelGGL(k_vgen<kVariantMont>, gg, dim3(256), 0, st, a);
  else
    hipLaunchKernelGGL(k_vgen<kVariantCrt>, gg, dim3(256), 0, st, a);
  return hipGetLastError() == hipSuccess ? RSAPRNG_OK : RSAPRNG_E_HIP;
}

}  // namespace rsaprng
