// A CPU stand-in for the part of the HIP runtime API that the library's host
// code (engine.cpp, host_pages.cpp, resident.cpp) uses, so that its queues,
// admission, tickets, scheduler and resident-engine ring can be built with
// g++ and run under ThreadSanitizer on a machine without a GPU.  TEST INFRASTRUCTURE ONLY: nothing in the library includes
// it; tests/test_scheduler_tsan_cpu.py puts this directory first on the
// include path of a separate host build.
//
// Semantics kept: a stream is an in-order queue served by its own thread;
// an event completes when the work recorded before it on its stream has
// run; "device" memory is host memory tracked in an allocation table so
// that pointer queries answer as the runtime would; graphs hold a memcpy
// node and a kernel node and replay them onto a stream.  Kernels are the
// functions of mock_kernels.cpp, which cipher pages with the C oracle.
#pragma once

#include <stddef.h>
#include <stdint.h>

typedef enum hipError_t {
  hipSuccess = 0,
  hipErrorInvalidValue = 1,
  hipErrorOutOfMemory = 2,
  hipErrorNotReady = 600,
  hipErrorUnknown = 999
} hipError_t;

typedef enum hipMemcpyKind {
  hipMemcpyHostToHost = 0,
  hipMemcpyHostToDevice = 1,
  hipMemcpyDeviceToHost = 2,
  hipMemcpyDeviceToDevice = 3,
  hipMemcpyDefault = 4
} hipMemcpyKind;

typedef enum hipMemoryType {
  hipMemoryTypeUnregistered = 0,
  hipMemoryTypeHost = 1,
  hipMemoryTypeDevice = 2
} hipMemoryType;

struct MockStream;
struct MockEvent;
struct MockGraph;
struct MockGraphExec;
struct MockGraphNode;
typedef MockStream* hipStream_t;
typedef MockEvent* hipEvent_t;
typedef MockGraph* hipGraph_t;
typedef MockGraphExec* hipGraphExec_t;
typedef MockGraphNode* hipGraphNode_t;
typedef void* hipDeviceptr_t;

struct dim3 {
  uint32_t x, y, z;
  dim3(uint32_t a = 1, uint32_t b = 1, uint32_t c = 1) : x(a), y(b), z(c) {}
};

struct hipDeviceProp_t {
  char name[256];
  char gcnArchName[256];
  int multiProcessorCount;
  int pciDomainID, pciBusID, pciDeviceID;
  size_t totalGlobalMem;
};

struct hipPointerAttribute_t {
  hipMemoryType type;
  int device;
  void* devicePointer;
  void* hostPointer;
  int isManaged;
  unsigned allocationFlags;
};

struct hipKernelNodeParams {
  dim3 blockDim;
  void** extra;
  void* func;
  dim3 gridDim;
  void** kernelParams;
  unsigned sharedMemBytes;
};

enum {
  hipStreamDefault = 0,
  hipStreamNonBlocking = 1,
  hipEventDefault = 0,
  hipEventDisableTiming = 2,
  hipHostMallocDefault = 0,
  hipHostMallocCoherent = 0x40000000
};

hipError_t hipGetDeviceCount(int* n);
hipError_t hipSetDevice(int d);
hipError_t hipGetDevice(int* d);
hipError_t hipGetDeviceProperties(hipDeviceProp_t* p, int d);
typedef enum hipDeviceAttribute_t {
  hipDeviceAttributeWallClockRate = 1
} hipDeviceAttribute_t;
hipError_t hipDeviceGetAttribute(int* v, hipDeviceAttribute_t a, int d);
hipError_t hipGetLastError();
hipError_t hipDeviceSynchronize();

hipError_t hipStreamCreate(hipStream_t* s);
hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned flags);
hipError_t hipStreamDestroy(hipStream_t s);
hipError_t hipStreamSynchronize(hipStream_t s);

hipError_t hipMalloc(void** p, size_t n);
hipError_t hipFree(void* p);
hipError_t hipHostMalloc(void** p, size_t n, unsigned flags);
hipError_t hipHostFree(void* p);
hipError_t hipMemset(void* p, int v, size_t n);
hipError_t hipMemsetAsync(void* p, int v, size_t n, hipStream_t s);
hipError_t hipMemcpy(void* dst, const void* src, size_t n, hipMemcpyKind k);
hipError_t hipMemcpyAsync(void* dst, const void* src, size_t n,
                          hipMemcpyKind k, hipStream_t s);
hipError_t hipPointerGetAttributes(hipPointerAttribute_t* a, const void* p);
hipError_t hipMemGetAddressRange(hipDeviceptr_t* base, size_t* size,
                                 hipDeviceptr_t p);

hipError_t hipEventCreate(hipEvent_t* e);
hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned flags);
hipError_t hipEventDestroy(hipEvent_t e);
hipError_t hipEventRecord(hipEvent_t e, hipStream_t s);
hipError_t hipEventQuery(hipEvent_t e);
hipError_t hipEventSynchronize(hipEvent_t e);
hipError_t hipEventElapsedTime(float* ms, hipEvent_t a, hipEvent_t b);
hipError_t hipStreamWaitEvent(hipStream_t s, hipEvent_t e, unsigned flags);

hipError_t hipGraphCreate(hipGraph_t* g, unsigned flags);
hipError_t hipGraphDestroy(hipGraph_t g);
hipError_t hipGraphAddMemcpyNode1D(hipGraphNode_t* n, hipGraph_t g,
                                   const hipGraphNode_t* deps, size_t ndeps,
                                   void* dst, const void* src, size_t count,
                                   hipMemcpyKind k);
hipError_t hipGraphAddKernelNode(hipGraphNode_t* n, hipGraph_t g,
                                 const hipGraphNode_t* deps, size_t ndeps,
                                 const hipKernelNodeParams* p);
hipError_t hipGraphInstantiate(hipGraphExec_t* e, hipGraph_t g, void* err,
                               char* log, size_t log_size);
hipError_t hipGraphExecDestroy(hipGraphExec_t e);
hipError_t hipGraphExecKernelNodeSetParams(hipGraphExec_t e, hipGraphNode_t n,
                                           const hipKernelNodeParams* p);
hipError_t hipGraphExecMemcpyNodeSetParams1D(hipGraphExec_t e,
                                             hipGraphNode_t n, void* dst,
                                             const void* src, size_t count,
                                             hipMemcpyKind k);
hipError_t hipGraphLaunch(hipGraphExec_t e, hipStream_t s);

// Test hooks (not HIP): run `fn` on stream `s` in order, as a kernel would;
// count of operations run so far on all streams.
#include <functional>
void mock_enqueue(hipStream_t s, std::function<void()> fn);
uint64_t mock_ops_run();
