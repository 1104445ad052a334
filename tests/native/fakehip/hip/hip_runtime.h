// A checking stand-in for the part of the HIP runtime API that the host
// library (host.cpp, server.cpp, noalloc.hip) calls, for host-only builds of
// that library under AddressSanitizer and UndefinedBehaviorSanitizer.  Device
// memory is host memory whose every range is checked against the live
// allocations; work on a stream is queued and runs later, in stream order
// (when the host waits on the stream, on an event, or frees memory), so a
// host-side reuse of a buffer that queued work still reads shows up as wrong
// data; stream capture records the queued operations into a graph that a
// launch replays.  The kernels are replaced by functions of the harness that
// check their arguments and write a tag of (instance, index) per output.
#pragma once
#include <stddef.h>
#include <stdint.h>

typedef int hipError_t;
enum {
  hipSuccess = 0,
  hipErrorInvalidValue = 1,
  hipErrorOutOfMemory = 2,
  hipErrorInvalidHandle = 400,
  hipErrorNotReady = 600,
  hipErrorStreamCaptureUnsupported = 900,
};
typedef struct FakeStream* hipStream_t;
typedef struct FakeEvent* hipEvent_t;
typedef struct FakeGraph* hipGraph_t;
typedef struct FakeGraphExec* hipGraphExec_t;
typedef void* hipGraphNode_t;
typedef enum {
  hipMemcpyHostToHost = 0,
  hipMemcpyHostToDevice = 1,
  hipMemcpyDeviceToHost = 2,
  hipMemcpyDeviceToDevice = 3,
  hipMemcpyDefault = 4
} hipMemcpyKind;
typedef enum {
  hipStreamCaptureModeGlobal = 0,
  hipStreamCaptureModeThreadLocal = 1,
  hipStreamCaptureModeRelaxed = 2
} hipStreamCaptureMode;
#define hipStreamNonBlocking 0x01
#define hipEventDisableTiming 0x02

typedef struct {
  char name[256];
  char gcnArchName[256];
  int multiProcessorCount;
} hipDeviceProp_t;

#define __device__
#define __global__
#define __host__
#define __align__(n) __attribute__((aligned(n)))

// A device symbol: its address and size, registered as device memory on the
// first hipGetSymbolAddress.
struct FakeSymbol {
  void* addr;
  size_t bytes;
};
#define HIP_SYMBOL(x) (FakeSymbol{(void*)&(x), sizeof(x)})

hipError_t hipGetDevice(int* dev);
hipError_t hipSetDevice(int dev);
hipError_t hipGetDeviceProperties(hipDeviceProp_t* prop, int dev);
hipError_t hipMalloc(void** p, size_t bytes);
hipError_t hipFree(void* p);
hipError_t hipHostMalloc(void** p, size_t bytes, unsigned flags);
hipError_t hipHostFree(void* p);
hipError_t hipMemcpy(void* dst, const void* src, size_t bytes, hipMemcpyKind kind);
hipError_t hipMemcpyAsync(void* dst, const void* src, size_t bytes, hipMemcpyKind kind,
                          hipStream_t s);
hipError_t hipMemset(void* p, int v, size_t bytes);
hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned flags);
hipError_t hipStreamDestroy(hipStream_t s);
hipError_t hipStreamSynchronize(hipStream_t s);
hipError_t hipStreamBeginCapture(hipStream_t s, hipStreamCaptureMode mode);
hipError_t hipStreamEndCapture(hipStream_t s, hipGraph_t* g);
hipError_t hipGraphInstantiate(hipGraphExec_t* e, hipGraph_t g, hipGraphNode_t* err_node,
                               char* log, size_t log_size);
hipError_t hipGraphLaunch(hipGraphExec_t e, hipStream_t s);
hipError_t hipGraphExecDestroy(hipGraphExec_t e);
hipError_t hipGraphDestroy(hipGraph_t g);
hipError_t hipEventCreate(hipEvent_t* e);
hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned flags);
hipError_t hipEventDestroy(hipEvent_t e);
hipError_t hipEventRecord(hipEvent_t e, hipStream_t s);
hipError_t hipEventSynchronize(hipEvent_t e);
hipError_t hipEventQuery(hipEvent_t e);
hipError_t hipEventElapsedTime(float* ms, hipEvent_t a, hipEvent_t b);
hipError_t hipGetSymbolAddress(void** p, FakeSymbol sym);
hipError_t hipDeviceSynchronize(void);

template <class T>
inline hipError_t hipMalloc(T** p, size_t bytes) {
  return hipMalloc(reinterpret_cast<void**>(p), bytes);
}
template <class T>
inline hipError_t hipHostMalloc(T** p, size_t bytes, unsigned flags) {
  return hipHostMalloc(reinterpret_cast<void**>(p), bytes, flags);
}

// ---- harness side --------------------------------------------------------
#include <functional>
namespace fakehip {
// Queue `op` on stream s (captured into the graph if s is capturing).
void enqueue(hipStream_t s, const char* what, std::function<void()> op);
// Whether [p, p + bytes) lies inside one live device allocation; on failure
// the run is reported and ends (exit status 3).
void need_device(const void* p, size_t bytes, const char* what);
bool is_device(const void* p, size_t bytes);
// Run every queued operation (all streams).
void drain();
// Live allocations and other counters, for leak checks at the end.
size_t live_device_allocations();
size_t live_streams();
size_t live_events();
}  // namespace fakehip
