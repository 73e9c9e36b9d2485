// A host-only stand-in for the part of the HIP runtime that the serving loop
// (hb_server.cpp) calls, for checking that loop on the CPU: streams are in-order op queues
// run by a thread each, events complete when their record op runs, waits block a stream
// until the recorded work they name is done, copies and "kernels" run on the host.  It
// also checks the rules a HIP program must keep with events and streams, and counts what
// is in flight (see fake_hip_report in fake_hip.hpp).
#pragma once

#include <stddef.h>
#include <stdint.h>

typedef enum hipError_t {
    hipSuccess = 0,
    hipErrorInvalidValue = 1,
    hipErrorOutOfMemory = 2,
    hipErrorNotReady = 600,
    hipErrorInvalidResourceHandle = 400,
} hipError_t;

typedef struct FakeStream *hipStream_t;
typedef struct FakeEvent *hipEvent_t;

typedef enum hipDeviceAttribute_t { hipDeviceAttributeMultiprocessorCount = 63 } hipDeviceAttribute_t;

enum hipMemcpyKind { hipMemcpyHostToHost = 0, hipMemcpyHostToDevice = 1, hipMemcpyDeviceToHost = 2,
                     hipMemcpyDeviceToDevice = 3, hipMemcpyDefault = 4 };

#define hipStreamNonBlocking 0x1u
#define hipEventDisableTiming 0x2u
#define hipHostMallocDefault 0x0u
#define hipHostMallocMapped 0x2u
#define hipHostMallocCoherent 0x40000000u

hipError_t hipSetDevice(int device);
hipError_t hipMalloc(void **ptr, size_t size);
hipError_t hipFree(void *ptr);
hipError_t hipHostMalloc(void **ptr, size_t size, unsigned int flags);
hipError_t hipHostFree(void *ptr);
hipError_t hipHostGetDevicePointer(void **dptr, void *hptr, unsigned int flags);
hipError_t hipStreamCreateWithFlags(hipStream_t *stream, unsigned int flags);
hipError_t hipStreamDestroy(hipStream_t stream);
hipError_t hipStreamSynchronize(hipStream_t stream);
hipError_t hipStreamWaitEvent(hipStream_t stream, hipEvent_t event, unsigned int flags);
hipError_t hipEventCreateWithFlags(hipEvent_t *event, unsigned int flags);
hipError_t hipEventDestroy(hipEvent_t event);
hipError_t hipEventRecord(hipEvent_t event, hipStream_t stream);
hipError_t hipEventQuery(hipEvent_t event);
hipError_t hipEventSynchronize(hipEvent_t event);
hipError_t hipMemcpyAsync(void *dst, const void *src, size_t n, hipMemcpyKind kind, hipStream_t stream);
hipError_t hipMemset(void *dst, int value, size_t n);
hipError_t hipDeviceGetAttribute(int *value, hipDeviceAttribute_t attr, int device);
const char *hipGetErrorString(hipError_t e);
