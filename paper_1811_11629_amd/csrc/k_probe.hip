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

// The store patterns of the chain-serial tile kernels: one work-group of WG
// lanes per 2^20-element chain, in steps of WG / 64 wave chunks of 1024
// elements; store j of a wave writes elements 128 j + 2 lane and the next of
// its chunk (1 KiB per store instruction), j = 0 .. 7, for c and for r, as
// 16-byte pairs, non-temporal (NT) or not.  SEQ: the wave's eight c stores,
// then its eight r stores (the kernels of 16 indices per lane, whose c and r
// take one transpose block in turn); otherwise c and r alternate (the kernels
// of two chunks of 8).  The values are the element indices.
typedef u64 u64x2 __attribute__((ext_vector_type(2)));

template <bool NT>
__device__ __forceinline__ void put2(u64* p, u64 a, u64 b) {
  if constexpr (NT)
    __builtin_nontemporal_store(u64x2{a, b}, reinterpret_cast<u64x2*>(p));
  else
    *reinterpret_cast<u64x2*>(p) = u64x2{a, b};
}

__device__ __forceinline__ u64 bits(u64 e) { return (u64)__double_as_longlong((double)e); }

template <int WG, bool NT, bool SEQ>
__global__ __launch_bounds__(WG) void k_probe_store_tile(u64* oc, double* orr) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const u64 chain0 = (u64)blockIdx.x << 20;
  u64* const r = reinterpret_cast<u64*>(orr);
  for (u64 step = 0; step < (1u << 20); step += (WG / 64) * 1024) {
    const u64 w0 = chain0 + step + (u64)wave * 1024 + 2 * lane;
    if constexpr (SEQ) {
#pragma unroll
      for (int j = 0; j < 8; ++j) put2<NT>(oc + w0 + j * 128, w0 + j * 128, w0 + j * 128 + 1);
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const u64 e = w0 + j * 128;
        put2<NT>(r + e, bits(e), bits(e + 1));
      }
    } else {
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const u64 e = w0 + j * 128;
        put2<NT>(oc + e, e, e + 1);
        put2<NT>(r + e, bits(e), bits(e + 1));
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
      hipLaunchKernelGGL((k_probe_store_tile<512, true, false>), dim3((unsigned)(n >> 20)),
                         dim3(512), 0, (hipStream_t)stream, out_u64, out_f64);
      return hipGetLastError() == hipSuccess ? RSAPRNG_OK : RSAPRNG_E_HIP;
    case RSAPRNG_PROBE_STORE_TILE_PLAIN:
      hipLaunchKernelGGL((k_probe_store_tile<512, false, false>), dim3((unsigned)(n >> 20)),
                         dim3(512), 0, (hipStream_t)stream, out_u64, out_f64);
      return hipGetLastError() == hipSuccess ? RSAPRNG_OK : RSAPRNG_E_HIP;
    case RSAPRNG_PROBE_STORE_BLOCK16:
      hipLaunchKernelGGL((k_probe_store_tile<256, true, true>), dim3((unsigned)(n >> 20)),
                         dim3(256), 0, (hipStream_t)stream, out_u64, out_f64);
      return hipGetLastError() == hipSuccess ? RSAPRNG_OK : RSAPRNG_E_HIP;
    case RSAPRNG_PROBE_STORE_BLOCK16_PLAIN:
      hipLaunchKernelGGL((k_probe_store_tile<256, false, true>), dim3((unsigned)(n >> 20)),
                         dim3(256), 0, (hipStream_t)stream, out_u64, out_f64);
      return hipGetLastError() == hipSuccess ? RSAPRNG_OK : RSAPRNG_E_HIP;
    case RSAPRNG_PROBE_STORE_LINEAR:
      hipLaunchKernelGGL(k_probe_store_linear, dim3(grid), dim3(256), 0, (hipStream_t)stream,
                         out_u64, out_f64, n);
      return hipGetLastError() == hipSuccess ? RSAPRNG_OK : RSAPRNG_E_HIP;
    default: return RSAPRNG_E_ARG;
  }
}

}  // namespace rsaprng
