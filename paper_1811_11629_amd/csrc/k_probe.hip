// Throughput probes behind the roofline figures: the issue rate of one VALU
// instruction class, and the store bandwidth of the tile kernels' output
// pattern.  They generate nothing; the benchmark times them to measure the
// ceilings that the generator's kernels are compared with.
#include <hip/hip_runtime.h>

#include "common.h"

namespace rsaprng {

namespace {

typedef uint64_t u64;
typedef uint32_t u32;

constexpr int kProbeWG = 256;    // 4 waves
constexpr int kProbeWGPerCU = 8;  // 32 waves per CU: 8 per SIMD
constexpr int kChains = 8;       // independent dependency chains per lane
constexpr int kUnroll = 4;       // rounds of kChains instructions per loop trip

// One instruction of the probed class on accumulator x or d (each depends on
// itself only, so the kChains chains of a lane are independent).  Mostly
// inline assembly, so that exactly that instruction is issued and the
// compiler cannot combine the unrolled copies.
template <int K>
__device__ __forceinline__ void op(u64& x, u32 m, double& d, double y) {
  if constexpr (K == RSAPRNG_PROBE_FMA_F64) {
    asm volatile("v_fma_f64 %0, %0, %1, %1" : "+v"(d) : "v"(y));
  } else if constexpr (K == RSAPRNG_PROBE_MUL_F64) {
    asm volatile("v_mul_f64 %0, %0, %1" : "+v"(d) : "v"(y));
  } else if constexpr (K == RSAPRNG_PROBE_ADD_F64) {
    asm volatile("v_add_f64 %0, %0, %1" : "+v"(d) : "v"(y));
  } else if constexpr (K == RSAPRNG_PROBE_RNDNE_F64) {
    asm volatile("v_rndne_f64 %0, %0" : "+v"(d));
  } else if constexpr (K == RSAPRNG_PROBE_MAD_U64_U32) {
    // written in C (the compiler emits exactly one v_mad_u64_u32; in inline
    // assembly its unused carry output made the compiler separate every pair
    // with a wait state)
    x = (u64)(u32)x * m + x;
  } else if constexpr (K == RSAPRNG_PROBE_MUL_LO_U32) {
    u32 v = (u32)x;
    asm volatile("v_mul_lo_u32 %0, %0, %1" : "+v"(v) : "v"(m));
    x = v;
  } else if constexpr (K == RSAPRNG_PROBE_MUL_HI_U32) {
    u32 v = (u32)x;
    asm volatile("v_mul_hi_u32 %0, %0, %1" : "+v"(v) : "v"(m));
    x = v;
  } else if constexpr (K == RSAPRNG_PROBE_ADD_U32) {
    u32 v = (u32)x;
    asm volatile("v_add_u32 %0, %0, %1" : "+v"(v) : "v"(m));
    x = v;
  } else if constexpr (K == RSAPRNG_PROBE_CVT_F64_U32) {
    // a dependent chain: the low word of d converted back into d
    d = (double)(u32)__double_as_longlong(d);
  } else if constexpr (K == RSAPRNG_PROBE_LSHL_ADD_U64) {
    asm volatile("v_lshl_add_u64 %0, %0, 0, %1" : "+v"(x) : "v"((u64)m));
  } else if constexpr (K == RSAPRNG_PROBE_MUL_U32_U24) {
    u32 v = (u32)x;
    asm volatile("v_mul_u32_u24 %0, %0, %1" : "+v"(v) : "v"(m));
    x = v;
  }
}

template <int K>
__global__ __launch_bounds__(kProbeWG) void k_probe_issue(u64 iters, u32 m, double y, u64* sink) {
  const u64 tid = (u64)blockIdx.x * kProbeWG + threadIdx.x;
  u64 x[kChains];
  double d[kChains];
#pragma unroll
  for (int c = 0; c < kChains; ++c) {
    x[c] = tid + c;
    d[c] = (double)(tid + c) * 0.5;
  }
  for (u64 it = 0; it < iters; ++it) {
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
#pragma unroll
      for (int c = 0; c < kChains; ++c) op<K>(x[c], m, d[c], y);
    }
  }
  u64 acc = 0;
#pragma unroll
  for (int c = 0; c < kChains; ++c) acc += x[c] ^ (u64)__double_as_longlong(d[c]);
  sink[tid] = acc;
}

// The store pattern of the chain-serial tile kernels: one work-group of 512
// lanes per 2^20-element chain, steps of 8192 elements, each wave storing two
// 512-element chunks per array per step as 16-byte non-temporal pairs (store
// j of a chunk writes elements 128 j + 2 lane and the next).  The values are
// the element indices.
typedef u64 u64x2 __attribute__((ext_vector_type(2)));

__global__ __launch_bounds__(512) void k_probe_store_tile(u64* oc, double* orr) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const u64 chain0 = (u64)blockIdx.x << 20;
  for (u64 step = 0; step < (1u << 20); step += 8192) {
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      const u64 chunk = chain0 + step + ((u64)wave * 2 + r) * 512;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const u64 e = chunk + (u64)j * 128 + 2 * lane;
        __builtin_nontemporal_store(u64x2{e, e + 1}, reinterpret_cast<u64x2*>(oc + e));
        __builtin_nontemporal_store(
            u64x2{(u64)__double_as_longlong((double)e), (u64)__double_as_longlong((double)(e + 1))},
            reinterpret_cast<u64x2*>(reinterpret_cast<u64*>(orr) + e));
      }
    }
  }
}

// A plain linear write of both arrays, 16 bytes per lane per store.
__global__ __launch_bounds__(256) void k_probe_store_linear(u64* oc, double* orr, u64 n) {
  const u64 stride = (u64)gridDim.x * 256 * 2;
  for (u64 e = ((u64)blockIdx.x * 256 + threadIdx.x) * 2; e < n; e += stride) {
    *reinterpret_cast<u64x2*>(oc + e) = u64x2{e, e + 1};
    *reinterpret_cast<u64x2*>(reinterpret_cast<u64*>(orr) + e) =
        u64x2{(u64)__double_as_longlong((double)e), (u64)__double_as_longlong((double)(e + 1))};
  }
}

template <int K>
int launch_issue(int grid, u64 iters, u64* sink, void* stream) {
  hipLaunchKernelGGL(k_probe_issue<K>, dim3(grid), dim3(kProbeWG), 0, (hipStream_t)stream, iters,
                     3u, 1.0000001, sink);
  return hipGetLastError() == hipSuccess ? RSAPRNG_OK : RSAPRNG_E_HIP;
}

}  // namespace

int probe_grid(int ncu) { return ncu * kProbeWGPerCU; }
u64 probe_threads(int ncu) { return (u64)probe_grid(ncu) * kProbeWG; }
u64 probe_ops_per_thread(u64 iters) { return iters * kUnroll * kChains; }

int launch_probe(int kind, int ncu, u64 n, u64* out_u64, double* out_f64, void* stream) {
  const int grid = probe_grid(ncu);
  switch (kind) {
    case RSAPRNG_PROBE_FMA_F64: return launch_issue<RSAPRNG_PROBE_FMA_F64>(grid, n, out_u64, stream);
    case RSAPRNG_PROBE_MUL_F64: return launch_issue<RSAPRNG_PROBE_MUL_F64>(grid, n, out_u64, stream);
    case RSAPRNG_PROBE_ADD_F64: return launch_issue<RSAPRNG_PROBE_ADD_F64>(grid, n, out_u64, stream);
    case RSAPRNG_PROBE_RNDNE_F64: return launch_issue<RSAPRNG_PROBE_RNDNE_F64>(grid, n, out_u64, stream);
    case RSAPRNG_PROBE_MAD_U64_U32: return launch_issue<RSAPRNG_PROBE_MAD_U64_U32>(grid, n, out_u64, stream);
    case RSAPRNG_PROBE_MUL_LO_U32: return launch_issue<RSAPRNG_PROBE_MUL_LO_U32>(grid, n, out_u64, stream);
    case RSAPRNG_PROBE_MUL_HI_U32: return launch_issue<RSAPRNG_PROBE_MUL_HI_U32>(grid, n, out_u64, stream);
    case RSAPRNG_PROBE_ADD_U32: return launch_issue<RSAPRNG_PROBE_ADD_U32>(grid, n, out_u64, stream);
    case RSAPRNG_PROBE_CVT_F64_U32: return launch_issue<RSAPRNG_PROBE_CVT_F64_U32>(grid, n, out_u64, stream);
    case RSAPRNG_PROBE_LSHL_ADD_U64: return launch_issue<RSAPRNG_PROBE_LSHL_ADD_U64>(grid, n, out_u64, stream);
    case RSAPRNG_PROBE_MUL_U32_U24: return launch_issue<RSAPRNG_PROBE_MUL_U32_U24>(grid, n, out_u64, stream);
    case RSAPRNG_PROBE_STORE_TILE:
      hipLaunchKernelGGL(k_probe_store_tile, dim3((unsigned)(n >> 20)), dim3(512), 0,
                         (hipStream_t)stream, out_u64, out_f64);
      return hipGetLastError() == hipSuccess ? RSAPRNG_OK : RSAPRNG_E_HIP;
    case RSAPRNG_PROBE_STORE_LINEAR:
      hipLaunchKernelGGL(k_probe_store_linear, dim3(grid), dim3(256), 0, (hipStream_t)stream,
                         out_u64, out_f64, n);
      return hipGetLastError() == hipSuccess ? RSAPRNG_OK : RSAPRNG_E_HIP;
    default: return RSAPRNG_E_ARG;
  }
}

}  // namespace rsaprng
