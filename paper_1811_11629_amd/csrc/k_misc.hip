// Small kernels (queue reset, statistics zero/finalise, test encryption) and
// the dispatch from a kernel shape to its tile-kernel family.
#include <algorithm>

#include "tiles.h"

namespace rsaprng {

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

template <int VAR>
__global__ void k_debug_encrypt(rsaprng_params P, const u64* m, u64* c, double* r, u64 count) {
  u64 i = blockIdx.x * (u64)blockDim.x + threadIdx.x;
  if (i >= count) return;
  double cd;
  u64 v = encrypt<VAR, 0>(m[i], P, cd);
  if (c) c[i] = v;
  if (r) r[i] = ratio(cd, P.nd);
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static int hip_rc(hipError_t e) { return e == hipSuccess ? RSAPRNG_OK : RSAPRNG_E_HIP; }

int launch_begin(DevCtl* ctl, void* stream) {
  hipLaunchKernelGGL(k_begin, dim3(1), dim3(1), 0, (hipStream_t)stream, ctl);
  return hip_rc(hipGetLastError());
}

int launch_mont_gen(const KernelShape&, const LaunchArgs&, void*, int*);
int launch_crt_gen(const KernelShape&, const LaunchArgs&, void*, int*);
int launch_mont_con(const KernelShape&, const LaunchArgs&, void*, int*);
int launch_crt_con(const KernelShape&, const LaunchArgs&, void*, int*);

static int dispatch(const KernelShape& s, const LaunchArgs* a, void* stream, int* occ) {
  static const LaunchArgs dummy{};
  const LaunchArgs& aa = a ? *a : dummy;
  if (s.variant == kVariantMont && s.mode == kModeGenerate) return launch_mont_gen(s, aa, stream, occ);
  if (s.variant == kVariantCrt && s.mode == kModeGenerate) return launch_crt_gen(s, aa, stream, occ);
  if (s.variant == kVariantMont && s.mode == kModeConsume) return launch_mont_con(s, aa, stream, occ);
  if (s.variant == kVariantCrt && s.mode == kModeConsume) return launch_crt_con(s, aa, stream, occ);
  return RSAPRNG_E_ARG;
}

int launch_tiles(const KernelShape& s, const LaunchArgs& a, void* stream) {
  return dispatch(s, &a, stream, nullptr);
}

int kernel_max_grid(const KernelShape& s, int* wg_per_cu) { return dispatch(s, nullptr, nullptr, wg_per_cu); }

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
