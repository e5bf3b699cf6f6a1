/*
 * Test double of the HIP runtime for host-only builds of the server
 * (tests/test_server_fake.py): the scheduler's own code, compiled with g++
 * against these declarations and linked with tests/fake_hip/fake_exec.cpp,
 * runs on the CPU with a simulated device.  Only what server.cpp and the
 * headers it includes use is declared.  Not part of the product library.
 */
#ifndef FFTCG_FAKE_HIP_RUNTIME_H
#define FFTCG_FAKE_HIP_RUNTIME_H

#include <stddef.h>

typedef enum {
    hipSuccess = 0,
    hipErrorInvalidValue = 1,
    hipErrorOutOfMemory = 2,
    hipErrorNotReady = 600,
} hipError_t;

typedef enum {
    hipMemcpyHostToHost = 0,
    hipMemcpyHostToDevice = 1,
    hipMemcpyDeviceToHost = 2,
    hipMemcpyDeviceToDevice = 3,
} hipMemcpyKind;

typedef enum {
    hipStreamCaptureModeGlobal = 0,
    hipStreamCaptureModeThreadLocal = 1,
    hipStreamCaptureModeRelaxed = 2,
} hipStreamCaptureMode;

struct FakeStream;
struct FakeEvent;
struct FakeGraph;
struct FakeGraphExec;
struct FakeGraphNode;
typedef FakeStream* hipStream_t;
typedef FakeEvent* hipEvent_t;
typedef FakeGraph* hipGraph_t;
typedef FakeGraphExec* hipGraphExec_t;
typedef FakeGraphNode* hipGraphNode_t;

#define hipHostMallocDefault 0x0u
#define hipHostMallocMapped 0x2u
#define hipHostMallocCoherent 0x40000000u
#define hipEventDisableTiming 0x2u
#define hipStreamNonBlocking 0x1u

hipError_t hipMallocRaw(void** p, size_t n);
template <class T>
inline hipError_t hipMalloc(T** p, size_t n) {
    return hipMallocRaw(reinterpret_cast<void**>(p), n);
}
hipError_t hipFree(void* p);
hipError_t hipHostMallocRaw(void** p, size_t n, unsigned flags);
template <class T>
inline hipError_t hipHostMalloc(T** p, size_t n, unsigned flags) {
    return hipHostMallocRaw(reinterpret_cast<void**>(p), n, flags);
}
hipError_t hipHostFree(void* p);
hipError_t hipHostGetDevicePointer(void** d, void* h, unsigned flags);
hipError_t hipMemcpy(void* dst, const void* src, size_t n, hipMemcpyKind k);
hipError_t hipMemcpyAsync(void* dst, const void* src, size_t n, hipMemcpyKind k, hipStream_t s);
hipError_t hipMemsetAsync(void* dst, int v, size_t n, hipStream_t s);
hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned flags);
hipError_t hipStreamSynchronize(hipStream_t s);
hipError_t hipStreamDestroy(hipStream_t s);
hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned flags);
hipError_t hipEventRecord(hipEvent_t e, hipStream_t s);
hipError_t hipEventQuery(hipEvent_t e);
hipError_t hipEventDestroy(hipEvent_t e);
hipError_t hipGetDeviceCount(int* n);
hipError_t hipSetDevice(int d);
hipError_t hipGetLastError();
hipError_t hipStreamBeginCapture(hipStream_t s, hipStreamCaptureMode mode);
hipError_t hipStreamEndCapture(hipStream_t s, hipGraph_t* g);
hipError_t hipGraphInstantiate(hipGraphExec_t* ex, hipGraph_t g, hipGraphNode_t* err, char* log, size_t n);
hipError_t hipGraphLaunch(hipGraphExec_t ex, hipStream_t s);
hipError_t hipGraphDestroy(hipGraph_t g);
hipError_t hipGraphExecDestroy(hipGraphExec_t ex);

#endif
