// Host-memory stand-in for the parts of the HIP runtime the lbrd host library
// calls (test infrastructure only).  The library's host code (validation,
// layouts, tilings, batch descriptors, the serving arena and scheduler) is
// compiled without device code and linked against this file, so that it runs
// on a machine without a GPU under AddressSanitizer and
// UndefinedBehaviorSanitizer:
//  - "device" memory is ordinary host memory of exactly the requested size,
//    so every copy, fill or staging the library does is bounds-checked;
//  - copies and fills run at once; streams, events and graphs are plain
//    host objects (events read a host clock);
//  - kernel launches run nothing: the launch configuration is checked
//    (grid and block sizes within the hardware's limits, dynamic LDS within
//    160 KB) and counted.
// Nothing here is part of the library.
#include <hip/hip_runtime_api.h>

#include <atomic>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>

namespace {

struct StubStream {
    bool capturing = false;
};
struct StubEvent {
    std::chrono::steady_clock::time_point t{};
    bool recorded = false;
};
struct StubGraph {
    int launches = 0;
};

std::atomic<long> g_launches{0};
std::atomic<long> g_bad_launches{0};
thread_local dim3 g_grid, g_block;
thread_local size_t g_shmem = 0;
thread_local hipStream_t g_stream = nullptr;

double now_ms(std::chrono::steady_clock::time_point t) {
    return std::chrono::duration<double, std::milli>(t.time_since_epoch()).count();
}

}  // namespace

extern "C" {

// ---- launches ---------------------------------------------------------------

hipError_t __hipPushCallConfiguration(dim3 grid, dim3 block, size_t shmem, hipStream_t stream) {
    g_grid = grid;
    g_block = block;
    g_shmem = shmem;
    g_stream = stream;
    return hipSuccess;
}

hipError_t __hipPopCallConfiguration(dim3 *grid, dim3 *block, size_t *shmem, hipStream_t *stream) {
    *grid = g_grid;
    *block = g_block;
    *shmem = g_shmem;
    *stream = g_stream;
    return hipSuccess;
}

hipError_t hipLaunchKernel(const void *fn, dim3 grid, dim3 block, void **args, size_t shmem, hipStream_t stream) {
    (void)stream;
    ++g_launches;
    const unsigned long long threads = (unsigned long long)block.x * block.y * block.z;
    const bool ok = fn && args && grid.x >= 1 && grid.y >= 1 && grid.z >= 1 && threads >= 1 && threads <= 1024 &&
                    shmem <= 160 * 1024;
    if (!ok) {
        ++g_bad_launches;
        std::fprintf(stderr, "stub: bad launch grid (%u %u %u) block (%u %u %u) lds %zu\n", grid.x, grid.y, grid.z,
                     block.x, block.y, block.z, shmem);
        return hipErrorInvalidConfiguration;
    }
    return hipSuccess;
}

void **__hipRegisterFatBinary(const void *) {
    static void *handle = nullptr;
    return &handle;
}
void __hipRegisterFunction(void **, const void *, char *, const char *, unsigned int, void *, void *, void *, void *,
                           int *) {}
void __hipUnregisterFatBinary(void **) {}
void __hipRegisterVar(void **, void *, char *, const char *, int, size_t, int, int) {}

// A __device__ variable's host stand-in has the variable's size here: its
// address serves as the "device" address.
hipError_t hipGetSymbolAddress(void **p, const void *symbol) {
    if (!p || !symbol) return hipErrorInvalidSymbol;
    *p = const_cast<void *>(symbol);
    return hipSuccess;
}

hipError_t hipFuncSetAttribute(const void *fn, hipFuncAttribute, int value) {
    return fn && value >= 0 && value <= 160 * 1024 ? hipSuccess : hipErrorInvalidValue;
}

hipError_t hipGetLastError(void) { return hipSuccess; }

const char *hipGetErrorString(hipError_t e) { return e == hipSuccess ? "hipSuccess" : "stub error"; }

// ---- device -------------------------------------------------------------------

hipError_t hipGetDevice(int *dev) {
    if (!dev) return hipErrorInvalidValue;
    *dev = 0;
    return hipSuccess;
}

hipError_t hipSetDevice(int dev) { return dev == 0 ? hipSuccess : hipErrorInvalidDevice; }

hipError_t hipDeviceGetAttribute(int *v, hipDeviceAttribute_t attr, int dev) {
    if (!v || dev != 0) return hipErrorInvalidValue;
    *v = attr == hipDeviceAttributeMultiprocessorCount ? 256 : 0;
    return hipSuccess;
}

hipError_t hipGetDevicePropertiesR0600(hipDeviceProp_tR0600 *prop, int dev) {
    if (!prop || dev != 0) return hipErrorInvalidValue;
    std::memset(prop, 0, sizeof(*prop));
    std::snprintf(prop->gcnArchName, sizeof(prop->gcnArchName), "gfx950");
    prop->multiProcessorCount = 256;
    return hipSuccess;
}

hipError_t hipDeviceSynchronize(void) { return hipSuccess; }

// ---- memory -------------------------------------------------------------------

hipError_t hipMalloc(void **p, size_t n) {
    if (!p) return hipErrorInvalidValue;
    void *q = nullptr;
    if (posix_memalign(&q, 256, n ? n : 1) != 0) return hipErrorOutOfMemory;
    std::memset(q, 0, n);
    *p = q;
    return hipSuccess;
}

hipError_t hipFree(void *p) {
    std::free(p);
    return hipSuccess;
}

hipError_t hipMemcpyAsync(void *dst, const void *src, size_t n, hipMemcpyKind, hipStream_t) {
    if (n && (!dst || !src)) return hipErrorInvalidValue;
    if (n) std::memmove(dst, src, n);
    return hipSuccess;
}

hipError_t hipMemcpy(void *dst, const void *src, size_t n, hipMemcpyKind kind) {
    return hipMemcpyAsync(dst, src, n, kind, nullptr);
}

hipError_t hipMemsetAsync(void *dst, int value, size_t n, hipStream_t) {
    if (n && !dst) return hipErrorInvalidValue;
    if (n) std::memset(dst, value, n);
    return hipSuccess;
}

// ---- streams, events, graphs --------------------------------------------------

hipError_t hipStreamCreateWithFlags(hipStream_t *s, unsigned int) {
    if (!s) return hipErrorInvalidValue;
    *s = reinterpret_cast<hipStream_t>(new StubStream());
    return hipSuccess;
}

hipError_t hipStreamCreate(hipStream_t *s) { return hipStreamCreateWithFlags(s, 0); }

hipError_t hipStreamDestroy(hipStream_t s) {
    delete reinterpret_cast<StubStream *>(s);
    return hipSuccess;
}

hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }

hipError_t hipStreamWaitEvent(hipStream_t, hipEvent_t e, unsigned int) {
    return e ? hipSuccess : hipErrorInvalidHandle;
}

hipError_t hipStreamBeginCapture(hipStream_t s, hipStreamCaptureMode) {
    if (!s) return hipErrorInvalidValue;
    reinterpret_cast<StubStream *>(s)->capturing = true;
    return hipSuccess;
}

hipError_t hipStreamEndCapture(hipStream_t s, hipGraph_t *g) {
    if (!s || !g) return hipErrorInvalidValue;
    StubStream *ss = reinterpret_cast<StubStream *>(s);
    if (!ss->capturing) return hipErrorIllegalState;
    ss->capturing = false;
    *g = reinterpret_cast<hipGraph_t>(new StubGraph());
    return hipSuccess;
}

hipError_t hipGraphInstantiate(hipGraphExec_t *exec, hipGraph_t g, hipGraphNode_t *, char *, size_t) {
    if (!exec || !g) return hipErrorInvalidValue;
    *exec = reinterpret_cast<hipGraphExec_t>(new StubGraph());
    return hipSuccess;
}

hipError_t hipGraphLaunch(hipGraphExec_t exec, hipStream_t) {
    if (!exec) return hipErrorInvalidValue;
    ++reinterpret_cast<StubGraph *>(exec)->launches;
    return hipSuccess;
}

hipError_t hipGraphDestroy(hipGraph_t g) {
    delete reinterpret_cast<StubGraph *>(g);
    return hipSuccess;
}

hipError_t hipGraphExecDestroy(hipGraphExec_t exec) {
    delete reinterpret_cast<StubGraph *>(exec);
    return hipSuccess;
}

hipError_t hipEventCreateWithFlags(hipEvent_t *e, unsigned) {
    if (!e) return hipErrorInvalidValue;
    *e = reinterpret_cast<hipEvent_t>(new StubEvent());
    return hipSuccess;
}

hipError_t hipEventCreate(hipEvent_t *e) { return hipEventCreateWithFlags(e, 0); }

hipError_t hipEventDestroy(hipEvent_t e) {
    delete reinterpret_cast<StubEvent *>(e);
    return hipSuccess;
}

hipError_t hipEventRecord(hipEvent_t e, hipStream_t) {
    if (!e) return hipErrorInvalidHandle;
    StubEvent *ev = reinterpret_cast<StubEvent *>(e);
    ev->t = std::chrono::steady_clock::now();
    ev->recorded = true;
    return hipSuccess;
}

hipError_t hipEventSynchronize(hipEvent_t e) { return e ? hipSuccess : hipErrorInvalidHandle; }

hipError_t hipEventElapsedTime(float *ms, hipEvent_t a, hipEvent_t b) {
    if (!ms || !a || !b) return hipErrorInvalidValue;
    const StubEvent *ea = reinterpret_cast<const StubEvent *>(a), *eb = reinterpret_cast<const StubEvent *>(b);
    if (!ea->recorded || !eb->recorded) return hipErrorNotReady;
    // a host clock: launches take no time here, so add a little per pair
    *ms = (float)(now_ms(eb->t) - now_ms(ea->t)) + 1e-3f;
    return hipSuccess;
}

// Counters for the driver: launches seen and launches refused.
long stub_launches(void) { return g_launches.load(); }
long stub_bad_launches(void) { return g_bad_launches.load(); }

}  // extern "C"
