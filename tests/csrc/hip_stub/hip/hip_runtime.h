/* Host-only stand-in for <hip/hip_runtime.h>: the types, constants and
 * runtime functions the library's host core (ca_api.cpp, ca_server.cpp)
 * uses, so that it can be compiled with g++ under AddressSanitizer and
 * UndefinedBehaviorSanitizer and driven without a GPU.  The functions are
 * implemented by the test harness (host_harness.cpp), which models device
 * memory as host memory, asynchronous work as completing some polls later,
 * and checks that no synchronous call is made where the caller forbids it.
 * Test infrastructure only. */
#pragma once

#include <stddef.h>
#include <stdint.h>

typedef enum hipError_t {
    hipSuccess = 0,
    hipErrorInvalidValue = 1,
    hipErrorOutOfMemory = 2,
    hipErrorNotReady = 600,
} hipError_t;

typedef struct ihipStream_t *hipStream_t;
typedef struct ihipEvent_t *hipEvent_t;
typedef struct ihipGraph_t *hipGraph_t;
typedef struct ihipGraphExec_t *hipGraphExec_t;
typedef struct ihipGraphNode_t *hipGraphNode_t;

typedef enum hipMemcpyKind {
    hipMemcpyHostToHost = 0,
    hipMemcpyHostToDevice = 1,
    hipMemcpyDeviceToHost = 2,
    hipMemcpyDeviceToDevice = 3,
    hipMemcpyDefault = 4,
} hipMemcpyKind;

typedef enum hipDeviceAttribute_t {
    hipDeviceAttributeMaxSharedMemoryPerBlock = 1,
    hipDeviceAttributeMultiprocessorCount = 2,
} hipDeviceAttribute_t;

typedef enum hipStreamCaptureMode {
    hipStreamCaptureModeGlobal = 0,
    hipStreamCaptureModeThreadLocal = 1,
    hipStreamCaptureModeRelaxed = 2,
} hipStreamCaptureMode;

#define hipStreamNonBlocking 0x01
#define hipEventDisableTiming 0x02

struct float4 {
    float x, y, z, w;
};
struct int4 {
    int x, y, z, w;
};
inline int4 make_int4(int x, int y, int z, int w) { return int4{x, y, z, w}; }

hipError_t hipGetDeviceCount(int *count);
hipError_t hipGetDevice(int *dev);
hipError_t hipSetDevice(int dev);
hipError_t hipDeviceGetAttribute(int *value, hipDeviceAttribute_t attr, int dev);
hipError_t hipDeviceSynchronize(void);
hipError_t hipGetLastError(void);

hipError_t hipMalloc(void **ptr, size_t bytes);
template <typename T>
hipError_t hipMalloc(T **ptr, size_t bytes)
{
    return hipMalloc(reinterpret_cast<void **>(ptr), bytes);
}
hipError_t hipFree(void *ptr);
hipError_t hipHostMalloc(void **ptr, size_t bytes, unsigned flags = 0);
template <typename T>
hipError_t hipHostMalloc(T **ptr, size_t bytes, unsigned flags = 0)
{
    return hipHostMalloc(reinterpret_cast<void **>(ptr), bytes, flags);
}
hipError_t hipHostFree(void *ptr);

hipError_t hipMemcpy(void *dst, const void *src, size_t bytes, hipMemcpyKind kind);
hipError_t hipMemcpyAsync(void *dst, const void *src, size_t bytes, hipMemcpyKind kind,
                          hipStream_t s);
hipError_t hipMemcpy2DAsync(void *dst, size_t dpitch, const void *src, size_t spitch,
                            size_t width, size_t height, hipMemcpyKind kind, hipStream_t s);
hipError_t hipMemset(void *dst, int value, size_t bytes);
hipError_t hipMemsetAsync(void *dst, int value, size_t bytes, hipStream_t s);

hipError_t hipStreamCreateWithFlags(hipStream_t *s, unsigned flags);
hipError_t hipStreamDestroy(hipStream_t s);
hipError_t hipStreamSynchronize(hipStream_t s);
hipError_t hipStreamWaitEvent(hipStream_t s, hipEvent_t e, unsigned flags);
hipError_t hipStreamBeginCapture(hipStream_t s, hipStreamCaptureMode mode);
hipError_t hipStreamEndCapture(hipStream_t s, hipGraph_t *graph);

hipError_t hipEventCreate(hipEvent_t *e);
hipError_t hipEventCreateWithFlags(hipEvent_t *e, unsigned flags);
hipError_t hipEventDestroy(hipEvent_t e);
hipError_t hipEventRecord(hipEvent_t e, hipStream_t s);
hipError_t hipEventQuery(hipEvent_t e);
hipError_t hipEventSynchronize(hipEvent_t e);
hipError_t hipEventElapsedTime(float *ms, hipEvent_t start, hipEvent_t stop);

hipError_t hipGraphInstantiate(hipGraphExec_t *exec, hipGraph_t graph, hipGraphNode_t *err_node,
                               char *log, size_t log_size);
hipError_t hipGraphLaunch(hipGraphExec_t exec, hipStream_t s);
hipError_t hipGraphExecDestroy(hipGraphExec_t exec);
hipError_t hipGraphDestroy(hipGraph_t graph);
