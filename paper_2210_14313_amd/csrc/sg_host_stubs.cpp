// Host-only build of the runtime (sg_api.cpp, sg_counts.cpp, sg_rules.cpp
// compiled with a host compiler under AddressSanitizer and
// UndefinedBehaviorSanitizer): a stand-in for the HIP runtime calls the host
// code makes, with "device" memory in the host heap, and kernel launchers
// that launch nothing.  The host logic -- validation, counts, rule tables,
// unranking, plan building and packing, the uploads (whose sizes the
// sanitizer checks against the allocations), graph capture bookkeeping,
// autotune and the plan-free entry points -- then runs on the CPU with no
// GPU.  Not part of libsgmdi.so; the results it leaves in output buffers
// are meaningless.
#include <hip/hip_runtime_api.h>

#include <atomic>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <unordered_set>

#include "sg_internal.hpp"
#include "sg_oscq.hpp"

namespace {
// Opaque handles: any distinct non-null address will do.
struct FakeHandle {
    int kind;
};
template <class H>
H make_handle(int kind)
{
    return reinterpret_cast<H>(new FakeHandle{kind});
}
void drop_handle(void* h) { delete static_cast<FakeHandle*>(h); }
int g_fail_countdown = 0;   // > 0: the allocation that brings it to 0 fails
std::mutex g_mu;
std::unordered_set<void*> g_live;   // "device" allocations not yet freed
std::atomic<long> g_launches{0};
int launched()
{
    ++g_launches;
    return 0;
}
}  // namespace

extern "C" {

hipError_t hipGetDevice(int* id)
{
    if (!id) return hipErrorInvalidValue;
    *id = 0;
    return hipSuccess;
}
hipError_t hipDeviceGetAttribute(int* pi, hipDeviceAttribute_t attr, int)
{
    if (!pi) return hipErrorInvalidValue;
    *pi = attr == hipDeviceAttributeMultiprocessorCount ? 256 : 0;
    return hipSuccess;
}
hipError_t hipGetDeviceProperties(hipDeviceProp_t* prop, int)
{
    if (!prop) return hipErrorInvalidValue;
    std::memset(prop, 0, sizeof *prop);
    std::strncpy(prop->gcnArchName, "host-stand-in", sizeof prop->gcnArchName - 1);
    prop->multiProcessorCount = 256;
    return hipSuccess;
}
hipError_t hipGetLastError(void) { return hipSuccess; }
const char* hipGetErrorString(hipError_t e) { return e == hipSuccess ? "no error" : "host-only build error"; }

hipError_t hipMalloc(void** ptr, size_t size)
{
    if (!ptr) return hipErrorInvalidValue;
    if (g_fail_countdown > 0 && --g_fail_countdown == 0) {
        *ptr = nullptr;
        return hipErrorOutOfMemory;
    }
    *ptr = std::malloc(size ? size : 1);
    if (!*ptr) return hipErrorOutOfMemory;
    std::lock_guard<std::mutex> lock(g_mu);
    g_live.insert(*ptr);
    return hipSuccess;
}
hipError_t hipFree(void* ptr)
{
    if (!ptr) return hipSuccess;
    {
        std::lock_guard<std::mutex> lock(g_mu);
        if (g_live.erase(ptr) != 1) return hipErrorInvalidValue;   // not from hipMalloc, or freed twice
    }
    std::free(ptr);
    return hipSuccess;
}

// Test hooks of the host-only build: allocations alive, launches made.
long sg_host_live_allocations(void)
{
    std::lock_guard<std::mutex> lock(g_mu);
    return (long)g_live.size();
}
long sg_host_launches(void) { return g_launches.load(); }
// The n-th allocation from now (1-based) fails with hipErrorOutOfMemory;
// n <= 0: none does.
void sg_host_fail_malloc_after(int n) { g_fail_countdown = n > 0 ? n : 0; }

hipError_t hipMemcpy(void* dst, const void* src, size_t n, hipMemcpyKind)
{
    if (n) std::memcpy(dst, src, n);
    return hipSuccess;
}
hipError_t hipMemcpyAsync(void* dst, const void* src, size_t n, hipMemcpyKind, hipStream_t)
{
    if (n) std::memcpy(dst, src, n);
    return hipSuccess;
}
hipError_t hipMemset(void* dst, int value, size_t n)
{
    if (n) std::memset(dst, value, n);
    return hipSuccess;
}
hipError_t hipMemsetAsync(void* dst, int value, size_t n, hipStream_t)
{
    if (n) std::memset(dst, value, n);
    return hipSuccess;
}

hipError_t hipEventCreate(hipEvent_t* ev)
{
    if (!ev) return hipErrorInvalidValue;
    *ev = make_handle<hipEvent_t>(1);
    return hipSuccess;
}
hipError_t hipEventRecord(hipEvent_t ev, hipStream_t) { return ev ? hipSuccess : hipErrorInvalidHandle; }
hipError_t hipEventSynchronize(hipEvent_t ev) { return ev ? hipSuccess : hipErrorInvalidHandle; }
hipError_t hipEventElapsedTime(float* ms, hipEvent_t a, hipEvent_t b)
{
    if (!ms || !a || !b) return hipErrorInvalidValue;
    *ms = 1.0f;
    return hipSuccess;
}
hipError_t hipEventDestroy(hipEvent_t ev)
{
    drop_handle(ev);
    return hipSuccess;
}

hipError_t hipStreamBeginCapture(hipStream_t s, hipStreamCaptureMode)
{
    return s ? hipSuccess : hipErrorInvalidValue;
}
hipError_t hipStreamEndCapture(hipStream_t s, hipGraph_t* g)
{
    if (!s || !g) return hipErrorInvalidValue;
    *g = make_handle<hipGraph_t>(2);
    return hipSuccess;
}
hipError_t hipGraphInstantiate(hipGraphExec_t* exec, hipGraph_t g, hipGraphNode_t*, char*, size_t)
{
    if (!exec || !g) return hipErrorInvalidValue;
    *exec = make_handle<hipGraphExec_t>(3);
    return hipSuccess;
}
hipError_t hipGraphLaunch(hipGraphExec_t exec, hipStream_t) { return exec ? hipSuccess : hipErrorInvalidValue; }
hipError_t hipGraphDestroy(hipGraph_t g)
{
    drop_handle(g);
    return hipSuccess;
}
hipError_t hipGraphExecDestroy(hipGraphExec_t exec)
{
    drop_handle(exec);
    return hipSuccess;
}

}  // extern "C"

namespace sg {

int launch_forward(int, int, int, const FwdWG*, unsigned int*, int, const double*, const float*, const double*,
                   double*, double*, void*)
{
    return launched();
}
int forward_capacity(int, int) { return 1 << 20; }
int launch_adjoint(int, bool, int, const WGDesc*, const ProbDev*, const double*, const float*, const double*,
                   const double*, double*, double*, void*)
{
    return launched();
}
int launch_unrank(int, int, uint64_t, uint64_t, int, const uint64_t*, int, int32_t*, int32_t*, int32_t*, void*)
{
    return launched();
}
const char* device_error_string(int) { return "host-only build"; }
int launch_one(int, int, int, int, int, int, const double*, double*, double*, double*, void*) { return launched(); }
int launch_points(int, const PointsLaunch&, void*) { return launched(); }
int launch_block_gather(const BlockSub*, int, int, const double*, double*, double*, void*) { return launched(); }
int launch_block_combine(const BlockProb*, int, const double*, const double*, const double*, const double*, double*, double*, void*)
{
    return launched();
}
int launch_oscq(int, int, int, int, int, int, const double*, const float*, const double*, double*, double*, double*,
                void*)
{
    return launched();
}
int launch_oscq_batch(int, int, const OscqDesc*, const double*, const float*, const double*, double*, double*, void*)
{
    return launched();
}
int launch_oscq_grad(int, const OscqDesc*, const double*, const double*, const double*, double*, double*, void*)
{
    return launched();
}

namespace {
double g_scratch[1 << 16];
}
int noalloc_scratch(double** ptr)
{
    *ptr = g_scratch;
    return 0;
}
int noalloc_launch(double*, int, int, int, int, int, const double*, double*, double*, void*) { return launched(); }
long noalloc_capacity_words() { return (long)(sizeof(g_scratch) / sizeof(double)); }

}  // namespace sg
