// Battery kernels: the fused battery of the CRT tile kernels (chain-serial
// family), and the battery of values already in device memory.
#include "tiles.h"

namespace rsaprng {

int launch_crt_bat(const KernelShape& s, const LaunchArgs& a, void* stream, int* occ) {
  return launch_family<kVariantCrt, kModeBattery>(s, a, stream, occ);
}

namespace {

// Battery of r[0 .. count), value j standing at index j.  A work-group takes
// whole units in turn: each block of 2^20 values is three units of 327680
// (one leading-bit collision trial, twenty urn trials of 2^14 values) and
// one of 65536 (four urn trials).  It walks a unit in steps of 8 WG values
// (a lane 8 consecutive, a wave 512), so the counts and their grouping are
// those of the fused battery.
template <int WG>
__global__ __launch_bounds__(WG) void k_battery_values(LaunchArgs a, const double* r, u64 count) {
  __shared__ TileShared<WG, kModeBattery> sh;
  const int lane = threadIdx.x & 63;
  const u32 wave = threadIdx.x >> 6;
  for (int i = threadIdx.x; i < kUrnWords; i += WG) sh.urn[i] = 0;
  for (int i = threadIdx.x; i < kBatLds; i += WG) sh.bh[i] = 0;
  __syncthreads();
  constexpr u64 kTrial = 1ull << kTrialLog2;
  constexpr u64 kStep = (u64)WG * 8;
  static_assert(kMsbTrial % kStep == 0 && kTrial % kStep == 0, "steps tile the units");
  const u64 last = count - 1;
  const u64 nunits = ((count + kBlock - 1) >> kBlockLog2) * 4;
  for (u64 u = blockIdx.x; u < nunits; u += gridDim.x) {
    const u64 blk = (u >> 2) << kBlockLog2;
    const u64 part = u & 3;
    const u64 ubase = blk + part * kMsbTrial;
    const u64 uend = part < 3 ? ubase + kMsbTrial : blk + kBlock;  // exclusive
    for (u64 s = ubase; s < uend && s < count; s += kStep) {
      const u64 laneStart = s + (u64)wave * 512 + (u64)lane * 8;
      double rv[8];
#pragma unroll
      for (int i = 0; i < 8; ++i) rv[i] = laneStart + i < count ? r[laneStart + i] : 0.0;
      battery_count<WG>(a, sh, 0, last, rv, laneStart);
      msb_step<WG>(a, sh, s, (u32)kStep, 0, last, blockIdx.x);
      // a step that ends an urn trial all of whose values exist (only the
      // data's last trial can be short, and it is its work-group's last)
      if (((s + kStep) & (kTrial - 1)) == 0 && s + kStep - 1 <= last) trial_flush<WG>(a, sh);
    }
  }
  battery_flush<WG>(a, sh);
}

}  // namespace

int launch_battery_values(const LaunchArgs& args, const double* r, uint64_t count, uint32_t slots,
                          void* stream) {
  constexpr int WG = 512;
  if (count == 0) return RSAPRNG_OK;
  if (!args.urn2 || slots == 0) return RSAPRNG_E_ARG;
  LaunchArgs a = args;
  a.tile_log2 = 12;  // steps of 8 WG values
  static_assert(8 * WG == 4096, "step size");
  const u64 nunits = ((count + kBlock - 1) >> kBlockLog2) * 4;
  int dev = 0, ncu = 0, blocks = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_battery_values<WG>, WG, 0) !=
          hipSuccess)
    return RSAPRNG_E_HIP;
  u64 grid = std::min<u64>(nunits, (u64)ncu * (blocks > 0 ? blocks : 1));
  grid = std::min<u64>(grid, slots);
  hipLaunchKernelGGL(k_battery_values<WG>, dim3((uint32_t)grid), dim3(WG), 0,
                     (hipStream_t)stream, a, r, count);
  return hipGetLastError() == hipSuccess ? RSAPRNG_OK : RSAPRNG_E_HIP;
}

}  // namespace rsaprng
