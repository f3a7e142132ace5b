// CPU stand-in for the HIP runtime calls the host driver makes: device memory
// is zeroed host memory, copies are memcpy, streams and events do nothing.
// Used only to run the host logic under AddressSanitizer without a GPU.
#pragma once
#include <cstdlib>
#include <cstring>
#include <cmath>
#include <cstdint>
#define __device__
#define __host__
#define __global__
#define __forceinline__ inline
#define __constant__ static
#define __shared__
#define __launch_bounds__(x)
typedef int hipError_t;
typedef struct ihipStream_t* hipStream_t;
typedef struct ihipEvent_t* hipEvent_t;
typedef struct ihipGraph_t* hipGraph_t;
typedef struct ihipGraphExec_t* hipGraphExec_t;
enum hipStreamCaptureMode { hipStreamCaptureModeGlobal = 0, hipStreamCaptureModeThreadLocal = 1, hipStreamCaptureModeRelaxed = 2 };
enum { hipSuccess = 0, hipMemcpyHostToDevice = 1, hipMemcpyDeviceToHost = 2, hipMemcpyDeviceToDevice = 3,
       hipStreamNonBlocking = 1 };
typedef int hipMemcpyKind;
struct dim3s { unsigned x, y, z; };
extern struct dim3s threadIdx, blockIdx, blockDim;
inline hipError_t hipMalloc(void** p, size_t n) { *p = calloc(1, n); return *p ? 0 : 2; }
inline hipError_t hipFree(void* p) { free(p); return 0; }
inline hipError_t hipGetDevice(int* d) { *d = 0; return 0; }
inline hipError_t hipMemGetInfo(size_t* f, size_t* t) { *f = *t = (size_t)1 << 34; return 0; }
inline hipError_t hipDeviceSynchronize() { return 0; }
#define hipHostMallocDefault 0u
inline hipError_t hipHostMalloc(void** p, size_t n, unsigned) { *p = calloc(1, n); return *p ? 0 : 2; }
inline hipError_t hipHostFree(void* p) { free(p); return 0; }
inline hipError_t hipMemcpyAsync(void* d, const void* s, size_t n, int, hipStream_t) { memcpy(d, s, n); return 0; }
inline hipError_t hipMemcpy(void* d, const void* s, size_t n, int) { memcpy(d, s, n); return 0; }
inline hipError_t hipMemsetAsync(void* d, int v, size_t n, hipStream_t) { memset(d, v, n); return 0; }
inline hipError_t hipStreamSynchronize(hipStream_t) { return 0; }
inline hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned) { *s = (hipStream_t)malloc(8); return 0; }
inline hipError_t hipStreamDestroy(hipStream_t s) { free(s); return 0; }
inline hipError_t hipStreamBeginCapture(hipStream_t, hipStreamCaptureMode) { return 0; }
inline hipError_t hipStreamEndCapture(hipStream_t, hipGraph_t* g) { *g = (hipGraph_t)malloc(8); return 0; }
inline hipError_t hipGraphInstantiate(hipGraphExec_t* e, hipGraph_t, void*, char*, size_t) { *e = (hipGraphExec_t)malloc(8); return 0; }
inline hipError_t hipGraphLaunch(hipGraphExec_t, hipStream_t) { return 0; }
inline hipError_t hipGraphExecDestroy(hipGraphExec_t e) { free(e); return 0; }
inline hipError_t hipGraphDestroy(hipGraph_t g) { free(g); return 0; }
inline hipError_t hipEventCreate(hipEvent_t* e) { *e = (hipEvent_t)malloc(8); return 0; }
inline hipError_t hipEventDestroy(hipEvent_t e) { free(e); return 0; }
inline hipError_t hipEventRecord(hipEvent_t, hipStream_t) { return 0; }
inline hipError_t hipEventSynchronize(hipEvent_t) { return 0; }
inline hipError_t hipEventElapsedTime(float* ms, hipEvent_t, hipEvent_t) { *ms = 0; return 0; }
inline hipError_t hipGetLastError() { return 0; }
inline const char* hipGetErrorString(hipError_t) { return "stub"; }
inline double __dsub_rn(double a, double b) { return a - b; }
inline double __dmul_rn(double a, double b) { return a * b; }
inline double __dadd_rn(double a, double b) { return a + b; }
inline double __shfl_xor(double v, int, int) { return v; }
inline void __syncthreads() {}
