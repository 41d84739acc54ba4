// Host-only mock of the HIP API subset used by lb_runtime.hip (CPU debugging only).
#pragma once
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <cstddef>
#include <cstdint>
typedef int hipError_t;
enum { hipSuccess = 0, hipErrorInvalidValue = 1 };
typedef struct MockStream* hipStream_t;
typedef struct MockEvent* hipEvent_t;
typedef struct MockGraph* hipGraph_t;
typedef struct MockGraph* hipGraphExec_t;
enum hipMemcpyKind { hipMemcpyHostToDevice, hipMemcpyDeviceToHost, hipMemcpyDeviceToDevice };
enum hipStreamCaptureMode { hipStreamCaptureModeThreadLocal };
#define hipStreamNonBlocking 1
#define hipEventDisableTiming 2
struct MockStream { int capturing; };
struct MockEvent { int x; int capture_gen; };
// Stream capture bookkeeping: an event recorded twice within one capture is reported (the
// runtime records each fork/join event once per capture).
inline int& mock_capture_gen() { static int g = 0; return g; }
inline int& mock_capturing() { static int c = 0; return c; }
struct MockGraph { int x; };
struct dim3 { unsigned x, y, z; dim3(unsigned a = 1, unsigned b = 1, unsigned c = 1) : x(a), y(b), z(c) {} };
#define __host__
#define __device__
#define __global__
#define __forceinline__ inline
#define __launch_bounds__(...)
#define __shared__
inline const char* hipGetErrorString(hipError_t) { return "mock error"; }
inline hipError_t hipGetLastError() { return hipSuccess; }
inline hipError_t hipMemcpyAsync(void* d, const void* s, size_t n, hipMemcpyKind, hipStream_t) { std::memcpy(d, s, n); return hipSuccess; }
inline hipError_t hipMemsetAsync(void* d, int v, size_t n, hipStream_t) { std::memset(d, v, n); return hipSuccess; }
inline hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
inline hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned) { *s = new MockStream{0}; return hipSuccess; }
inline hipError_t hipStreamDestroy(hipStream_t s) { delete s; return hipSuccess; }
inline hipError_t hipEventCreate(hipEvent_t* e) { *e = new MockEvent{0, -1}; return hipSuccess; }
inline hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned) { *e = new MockEvent{0, -1}; return hipSuccess; }
inline hipError_t hipEventDestroy(hipEvent_t e) { delete e; return hipSuccess; }
inline hipError_t hipEventRecord(hipEvent_t e, hipStream_t) {
    if (mock_capturing()) {
        if (e->capture_gen == mock_capture_gen()) {
            std::fprintf(stderr, "mock: event recorded twice within one capture\n");
            std::abort();
        }
        e->capture_gen = mock_capture_gen();
    }
    e->x++;
    return hipSuccess;
}
inline hipError_t hipEventSynchronize(hipEvent_t) { return hipSuccess; }
inline hipError_t hipEventElapsedTime(float* t, hipEvent_t, hipEvent_t) { *t = 1.f; return hipSuccess; }
inline hipError_t hipStreamWaitEvent(hipStream_t, hipEvent_t e, unsigned) { return e ? hipSuccess : hipErrorInvalidValue; }
inline hipError_t hipStreamBeginCapture(hipStream_t s, hipStreamCaptureMode) {
    s->capturing = 1;
    mock_capturing() = 1;
    ++mock_capture_gen();
    return hipSuccess;
}
inline hipError_t hipStreamEndCapture(hipStream_t s, hipGraph_t* g) {
    s->capturing = 0;
    mock_capturing() = 0;
    *g = new MockGraph{0};
    return hipSuccess;
}
inline hipError_t hipGraphInstantiate(hipGraphExec_t* e, hipGraph_t, void*, void*, size_t) { *e = new MockGraph{0}; return hipSuccess; }
inline hipError_t hipGraphLaunch(hipGraphExec_t, hipStream_t) { return hipSuccess; }
inline hipError_t hipGraphUpload(hipGraphExec_t e, hipStream_t) { return e ? hipSuccess : hipErrorInvalidValue; }
inline hipError_t hipGraphExecDestroy(hipGraphExec_t e) { delete e; return hipSuccess; }
inline hipError_t hipGraphDestroy(hipGraph_t g) { delete g; return hipSuccess; }
#define hipLaunchKernelGGL(k, g, b, sh, st, ...) ((void)0)
#define hipExtLaunchKernelGGL(k, g, b, sh, st, e0, e1, fl, ...) ((void)0)
