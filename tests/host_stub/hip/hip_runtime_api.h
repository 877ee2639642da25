// A stand-in for the HIP runtime API, for building the library's host code on
// a machine without a GPU: handles are heap objects owned by the stub
// (tests/host_stub/stub_runtime.cpp), device pointers are addresses in a
// reserved range that is never dereferenced, and every call checks the
// lifetime and capture rules of the real runtime.  Only what the host code of
// the library uses is declared.
#pragma once
#include <stddef.h>
#include <stdint.h>

typedef enum hipError_t {
  hipSuccess = 0,
  hipErrorInvalidValue = 1,
  hipErrorOutOfMemory = 2,
  hipErrorInvalidResourceHandle = 400,
  hipErrorStreamCaptureUnsupported = 900,
  hipErrorStreamCaptureInvalidated = 901,
  hipErrorStreamCaptureUnjoined = 904,
  hipErrorStreamCaptureIsolation = 905,
  hipErrorUnknown = 999
} hipError_t;

typedef struct StubStream* hipStream_t;
typedef struct StubEvent* hipEvent_t;
typedef struct StubGraph* hipGraph_t;
typedef struct StubExec* hipGraphExec_t;
typedef struct StubNode* hipGraphNode_t;
typedef int hipDevice_t;

typedef enum hipMemcpyKind {
  hipMemcpyHostToHost = 0,
  hipMemcpyHostToDevice = 1,
  hipMemcpyDeviceToHost = 2,
  hipMemcpyDeviceToDevice = 3,
  hipMemcpyDefault = 4
} hipMemcpyKind;

typedef enum hipStreamCaptureMode {
  hipStreamCaptureModeGlobal = 0,
  hipStreamCaptureModeThreadLocal = 1,
  hipStreamCaptureModeRelaxed = 2
} hipStreamCaptureMode;

typedef enum hipStreamCaptureStatus {
  hipStreamCaptureStatusNone = 0,
  hipStreamCaptureStatusActive = 1,
  hipStreamCaptureStatusInvalidated = 2
} hipStreamCaptureStatus;

#define hipEventDefault 0x0u
#define hipEventDisableTiming 0x2u
#define hipStreamDefault 0x0u
#define hipStreamNonBlocking 0x1u

#ifdef __cplusplus
extern "C" {
#endif
hipError_t hipGetDevice(int* device);
hipError_t hipStreamGetDevice(hipStream_t stream, hipDevice_t* device);
hipError_t hipGetLastError(void);
hipError_t hipStreamCreateWithFlags(hipStream_t* stream, unsigned int flags);
hipError_t hipStreamDestroy(hipStream_t stream);
hipError_t hipStreamSynchronize(hipStream_t stream);
hipError_t hipStreamWaitEvent(hipStream_t stream, hipEvent_t event, unsigned int flags);
hipError_t hipStreamBeginCapture(hipStream_t stream, hipStreamCaptureMode mode);
hipError_t hipStreamEndCapture(hipStream_t stream, hipGraph_t* graph);
hipError_t hipStreamIsCapturing(hipStream_t stream, hipStreamCaptureStatus* status);
hipError_t hipEventCreate(hipEvent_t* event);
hipError_t hipEventCreateWithFlags(hipEvent_t* event, unsigned flags);
hipError_t hipEventRecord(hipEvent_t event, hipStream_t stream);
hipError_t hipEventDestroy(hipEvent_t event);
hipError_t hipEventSynchronize(hipEvent_t event);
hipError_t hipEventElapsedTime(float* ms, hipEvent_t start, hipEvent_t stop);
hipError_t hipGraphInstantiate(hipGraphExec_t* exec, hipGraph_t graph, hipGraphNode_t* error_node,
                               char* log, size_t log_size);
hipError_t hipGraphDestroy(hipGraph_t graph);
hipError_t hipGraphExecDestroy(hipGraphExec_t exec);
hipError_t hipGraphLaunch(hipGraphExec_t exec, hipStream_t stream);
hipError_t hipMemcpyAsync(void* dst, const void* src, size_t bytes, hipMemcpyKind kind, hipStream_t stream);
hipError_t hipGetSymbolAddress(void** dev_ptr, const void* symbol);
#ifdef __cplusplus
}
#endif
