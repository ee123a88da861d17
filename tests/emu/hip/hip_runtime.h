// Host emulation of the HIP primitives that the BOS kernels use -- TEST
// INFRASTRUCTURE ONLY. A workgroup runs as one host thread per work-item
// (blocks one after another), __syncthreads is a barrier over the block,
// cross-lane operations exchange through a per-wave array between wave
// barriers, device memory is host memory, and a captured graph is a list of
// launches replayed in order. It lets the kernels' logic (indexing, barriers,
// LDS layout, termination) be checked on a machine without a GPU; it says
// nothing about the GPU runtime or timing.
#pragma once
#include <atomic>
#include <barrier>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <memory>
#include <thread>
#include <vector>

#define __global__
#define __device__
#define __host__
#define __forceinline__ inline
#define __launch_bounds__(...)
#define __shared__ static

struct dim3 {
    unsigned x, y, z;
    dim3(unsigned a = 1, unsigned b = 1, unsigned c = 1) : x(a), y(b), z(c) {}
};
extern thread_local dim3 threadIdx, blockIdx;
extern dim3 blockDim, gridDim;
extern void* emu_dyn_lds;
extern std::barrier<>* emu_block_bar;
extern std::barrier<>* emu_wave_bar[16];
extern unsigned long long emu_xchg[16][64];

inline void __syncthreads() { emu_block_bar->arrive_and_wait(); }
inline void emu_wave_sync() { emu_wave_bar[threadIdx.x / 64]->arrive_and_wait(); }
template <typename T>
T emu_shfl(T v, int src) {
    static_assert(sizeof(T) <= 8, "");
    const int w = threadIdx.x / 64, l = threadIdx.x % 64;
    unsigned long long u = 0;
    std::memcpy(&u, &v, sizeof(T));
    emu_wave_sync();
    emu_xchg[w][l] = u;
    emu_wave_sync();
    unsigned long long r = emu_xchg[w][((src % 64) + 64) % 64];
    emu_wave_sync();
    T o;
    std::memcpy(&o, &r, sizeof(T));
    return o;
}
template <typename T>
T __shfl(T v, int src, int = 64) { return emu_shfl(v, src); }
template <typename T>
T __shfl_xor(T v, int m, int = 64) { return emu_shfl(v, (int)(threadIdx.x % 64) ^ m); }
inline int atomicAdd(int* p, int v) { return __atomic_fetch_add(p, v, __ATOMIC_SEQ_CST); }
inline unsigned long long atomicMax(unsigned long long* p, unsigned long long v) {
    unsigned long long o = __atomic_load_n(p, __ATOMIC_SEQ_CST);
    while (o < v && !__atomic_compare_exchange_n(p, &o, v, false, __ATOMIC_SEQ_CST, __ATOMIC_SEQ_CST)) {
    }
    return o;
}
inline int atomicOr(int* p, int v) { return __atomic_fetch_or(p, v, __ATOMIC_SEQ_CST); }
#define __HIP_MEMORY_SCOPE_SYSTEM 5
#define __hip_atomic_load(p, order, scope) __atomic_load_n((p), (order))
inline float emu_fmed3f(float a, float b, float c) { return std::fmax(std::fmin(a, b), std::fmin(std::fmax(a, b), c)); }
#define __builtin_amdgcn_fmed3f emu_fmed3f
#define __builtin_amdgcn_fence(a, b) ((void)0)
#define __builtin_amdgcn_wave_barrier() emu_wave_sync()
// readfirstlane: the value of the wave's first lane (lane 0 is always active
// where the kernels use it; a differing value would be a kernel bug)
inline int emu_readfirstlane(int v) {
    const int r = emu_shfl(v, 0);
    if (r != v) {
        std::fprintf(stderr, "readfirstlane of a non-uniform value\n");
        std::abort();
    }
    return r;
}
#define __builtin_amdgcn_readfirstlane emu_readfirstlane

typedef int hipError_t;
enum { hipSuccess = 0, hipErrorInvalidValue = 1, hipErrorNotReady = 600 };
typedef void* hipStream_t;
typedef void* hipEvent_t;
typedef struct EmuGraph* hipGraph_t;
typedef struct EmuGraph* hipGraphExec_t;
enum hipMemcpyKind { hipMemcpyHostToDevice, hipMemcpyDeviceToHost, hipMemcpyDeviceToDevice, hipMemcpyHostToHost };
enum { hipHostMallocMapped = 0x2, hipHostMallocCoherent = 0x40000000 };
enum { hipStreamNonBlocking = 1, hipStreamCaptureModeThreadLocal = 1, hipFuncAttributeMaxDynamicSharedMemorySize = 8,
       hipEventDisableTiming = 2 };
typedef int hipStreamCaptureMode;

struct EmuGraph {
    std::vector<std::function<void()>> nodes;
};
extern hipStream_t emu_capturing;
extern EmuGraph* emu_graph;

void emu_run(dim3 g, dim3 b, size_t lds, std::function<void()> body);
template <typename F>
inline void emu_launch(dim3 g, dim3 b, size_t lds, hipStream_t s, F body) {
    if (s != nullptr && s == emu_capturing) {
        emu_graph->nodes.push_back([=]() { emu_run(g, b, lds, body); });
    } else {
        emu_run(g, b, lds, body);
    }
}

inline const char* hipGetErrorString(hipError_t) { return "emulated error"; }
inline hipError_t hipGetLastError() { return hipSuccess; }
inline hipError_t hipMalloc(void** p, size_t n) { *p = std::calloc(n ? n : 1, 1); return hipSuccess; }
template <typename T>
inline hipError_t hipMalloc(T** p, size_t n) { return hipMalloc((void**)p, n); }
inline hipError_t hipFree(void* p) { std::free(p); return hipSuccess; }
inline hipError_t hipHostMalloc(void** p, size_t n, unsigned) { *p = std::calloc(n ? n : 1, 1); return hipSuccess; }
inline hipError_t hipHostFree(void* p) { std::free(p); return hipSuccess; }
inline hipError_t hipHostGetDevicePointer(void** d, void* h, unsigned) { *d = h; return hipSuccess; }
inline hipError_t hipMemcpy(void* d, const void* s, size_t n, hipMemcpyKind) { std::memcpy(d, s, n); return hipSuccess; }
inline hipError_t hipMemcpyAsync(void* d, const void* s, size_t n, hipMemcpyKind, hipStream_t) { std::memcpy(d, s, n); return hipSuccess; }
inline hipError_t hipMemsetAsync(void* d, int v, size_t n, hipStream_t) { std::memset(d, v, n); return hipSuccess; }
inline hipError_t hipMemset(void* d, int v, size_t n) { std::memset(d, v, n); return hipSuccess; }
inline hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
inline hipError_t hipDeviceSynchronize() { return hipSuccess; }
inline hipError_t hipFuncSetAttribute(const void*, int, int) { return hipSuccess; }
inline hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned) { *s = std::malloc(1); return hipSuccess; }
inline hipError_t hipStreamDestroy(hipStream_t s) { std::free(s); return hipSuccess; }
inline hipError_t hipStreamBeginCapture(hipStream_t s, int) { emu_capturing = s; emu_graph = new EmuGraph(); return hipSuccess; }
inline hipError_t hipStreamEndCapture(hipStream_t, hipGraph_t* g) { *g = emu_graph; emu_capturing = nullptr; emu_graph = nullptr; return hipSuccess; }
inline hipError_t hipGraphInstantiate(hipGraphExec_t* e, hipGraph_t g, void*, void*, size_t) { *e = g; return hipSuccess; }
inline hipError_t hipGraphLaunch(hipGraphExec_t e, hipStream_t) { for (auto& n : e->nodes) n(); return hipSuccess; }
inline hipError_t hipGraphExecDestroy(hipGraphExec_t) { return hipSuccess; }
// launches run to completion when enqueued, so an event is complete at once
inline hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned) { *e = std::malloc(1); return hipSuccess; }
inline hipError_t hipEventRecord(hipEvent_t, hipStream_t) { return hipSuccess; }
inline hipError_t hipEventQuery(hipEvent_t) { return hipSuccess; }
inline hipError_t hipEventDestroy(hipEvent_t e) { std::free(e); return hipSuccess; }
inline hipError_t hipGraphDestroy(hipGraph_t g) { delete g; return hipSuccess; }
struct alignas(8) float2 { float x, y; };
struct alignas(16) float4 { float x, y, z, w; };
struct alignas(16) uint4 { unsigned x, y, z, w; };
inline float2 make_float2(float a, float b) { return float2{a, b}; }
using std::min;
using std::max;
