// Battery kernels: the fused battery of the CRT tile kernels (chain-serial
// family), and the battery of values already in device memory.
#include "tiles.h"

namespace rsaprng {

int launch_crt_bat(const KernelShape& s, const LaunchArgs& a, void* stream, int* occ) {
  return launch_family<kVariantCrt, kModeBattery>(s, a, stream, occ);
}

namespace {

// Battery of r[0 .. count), value j standing at index j.  A work-group takes
// whole collision trials (aligned blocks of 2^14 values) in turn, walking each
// in steps of 8 WG values (a lane 8 consecutive, a wave 512), so the counts
// and their grouping are those of the fused battery.
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
  const u64 last = count - 1;
  const u64 ntrials = (count + kTrial - 1) >> kTrialLog2;
  for (u64 t = blockIdx.x; t < ntrials; t += gridDim.x) {
    const u64 base = t << kTrialLog2;
    for (u64 s = base; s < base + kTrial && s < count; s += kStep) {
      const u64 laneStart = s + (u64)wave * 512 + (u64)lane * 8;
      double rv[8];
#pragma unroll
      for (int i = 0; i < 8; ++i) rv[i] = laneStart + i < count ? r[laneStart + i] : 0.0;
      battery_count<WG>(a, sh, 0, last, rv, laneStart);
    }
    if (base + kTrial - 1 <= last) trial_flush<WG>(a, sh);
  }
  battery_flush<WG>(a, sh);
}

}  // namespace

int launch_battery_values(const LaunchArgs& a, const double* r, uint64_t count, void* stream) {
  constexpr int WG = 512;
  if (count == 0) return RSAPRNG_OK;
  const u64 ntrials = (count + (1ull << kTrialLog2) - 1) >> kTrialLog2;
  int dev = 0, ncu = 0, blocks = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_battery_values<WG>, WG, 0) !=
          hipSuccess)
    return RSAPRNG_E_HIP;
  const u64 grid = std::min<u64>(ntrials, (u64)ncu * (blocks > 0 ? blocks : 1));
  hipLaunchKernelGGL(k_battery_values<WG>, dim3((uint32_t)grid), dim3(WG), 0,
                     (hipStream_t)stream, a, r, count);
  return hipGetLastError() == hipSuccess ? RSAPRNG_OK : RSAPRNG_E_HIP;
}

}  // namespace rsaprng
