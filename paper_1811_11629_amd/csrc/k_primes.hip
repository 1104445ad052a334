// Parameter generation on the device: counting primes or safe primes in a
// range, and finding the next prime (safe if asked, with an exponent filter)
// at or above each of many draws (Implementation section).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "common.h"
#include "primes.h"

namespace rsaprng {

namespace {

// Numbers in [lo, hi) coprime to 30, one wheel row of 30 per thread and step.
__global__ __launch_bounds__(256) void k_count_primes(uint64_t row0, uint64_t nrows, uint64_t lo,
                                                      uint64_t hi, int safe, SmallPrimeTable sp,
                                                      unsigned long long* count) {
  uint32_t c = 0;
  for (uint64_t row = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; row < nrows;
       row += (uint64_t)gridDim.x * blockDim.x)
    c += count_row(row0 + row, lo, hi, safe != 0, sp);
  if (blockIdx.x == 0 && threadIdx.x == 0) c += count_small(lo, hi, safe != 0);
#pragma unroll
  for (int m = 1; m < 64; m <<= 1) c += __shfl_xor(c, m, 64);
  if ((threadIdx.x & 63) == 0 && c) atomicAdd(count, (unsigned long long)c);
}

__global__ void k_zero_u64(unsigned long long* p) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *p = 0;
}

struct NextArgs {
  const uint64_t* x;
  uint64_t* out;
  uint64_t n;
  uint64_t span;
  int safe;
  int nexp;
  uint32_t exps[8];
  SmallPrimeTable sp;
};

// Smallest qualifying p in [x, min(x + span, 2^32)), else 0.
__global__ __launch_bounds__(256) void k_next_primes(NextArgs a) {
  const uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  if (i >= a.n) return;
  const uint64_t x = a.x[i];
  const uint64_t end = x + a.span < (1ull << 32) ? x + a.span : (1ull << 32);
  uint64_t found = 0;
  for (uint64_t p = x; p < end; ++p) {
    if (p > 2 && (p & 1) == 0) continue;
    bool ok = true;
    for (int f = 0; f < a.nexp; ++f) ok = ok && (p % a.exps[f] != 1);
    if (ok && candidate_ok((uint32_t)p, a.safe != 0, a.sp)) {
      found = p;
      break;
    }
  }
  a.out[i] = found;
}

}  // namespace

int launch_count_primes(uint64_t lo, uint64_t hi, int safe, unsigned long long* count_dev,
                        void* stream) {
  hipStream_t st = (hipStream_t)stream;
  hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, st, count_dev);
  if (hipGetLastError() != hipSuccess) return RSAPRNG_E_HIP;
  if (lo >= hi) return RSAPRNG_OK;
  const uint64_t row0 = lo / 30, row1 = (hi + 29) / 30;
  const uint64_t nrows = row1 - row0;
  const uint64_t grid = std::min<uint64_t>((nrows + 255) / 256, 4096);
  hipLaunchKernelGGL(k_count_primes, dim3((uint32_t)grid), dim3(256), 0, st, row0, nrows, lo, hi,
                     safe, make_small_primes(), count_dev);
  return hipGetLastError() == hipSuccess ? RSAPRNG_OK : RSAPRNG_E_HIP;
}

int launch_next_primes(const uint64_t* x, uint64_t n, int safe, const uint32_t* exps, int nexp,
                       uint64_t span, uint64_t* out, void* stream) {
  if (n == 0) return RSAPRNG_OK;
  NextArgs a;
  a.x = x;
  a.out = out;
  a.n = n;
  a.span = span;
  a.safe = safe;
  a.nexp = nexp;
  for (int i = 0; i < 8; ++i) a.exps[i] = i < nexp ? exps[i] : 1u;
  a.sp = make_small_primes();
  const uint64_t grid = (n + 255) / 256;
  hipLaunchKernelGGL(k_next_primes, dim3((uint32_t)grid), dim3(256), 0, (hipStream_t)stream, a);
  return hipGetLastError() == hipSuccess ? RSAPRNG_OK : RSAPRNG_E_HIP;
}

}  // namespace rsaprng
