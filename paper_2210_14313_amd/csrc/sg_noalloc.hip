// sg_integrate_noalloc: the plan-free path for callers that cannot allocate
// device memory (code under HIP graph capture, tight serving loops).
//
// The split launches of sg_integrate (k_one, k_oscq with G > 1 workgroups)
// need scratch for the workgroups' partials and an arrival counter.  Here it
// is a fixed array in device memory that the library's code object carries:
// each GPU the library runs on holds its own copy until the process ends.
// Its address is taken once per device with hipGetSymbolAddress (at context
// creation, with that device current) and passed to the kernels like any
// other buffer; host code never uses the array's name as an address.  The
// counter starts at zero when the code object is loaded and every completed
// launch leaves it at zero.  Every call on one GPU shares the array, so calls
// that overlap in time on one GPU race (results undefined).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>

#include "sg_internal.hpp"
#include "sg_oscq.hpp"

namespace sg {

// Doubles of the array: the counter block and kOneMaxG partials of the
// larger of the two partial layouts (real sweep, complex sweep).
constexpr int kNoAllocWords = kOneHead + kOneMaxG * (kOneWords > kOscqWords ? kOneWords : kOscqWords);
static_assert(kOneHead == kOscqScratchHead, "one counter block for both sweeps");
static __device__ __align__(256) double scratch[kNoAllocWords];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_mu;
double* g_ptr[kMaxDevices] = {};
}  // namespace

// Address of the current device's scratch array (looked up once per device).
// Returns 0 or the HIP error code.
int noalloc_scratch(double** ptr)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return (int)e;
    if (dev < 0 || dev >= kMaxDevices) return (int)hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return (int)e;
        g_ptr[dev] = static_cast<double*>(p);
    }
    *ptr = g_ptr[dev];
    return 0;
}

// Split launch of one integrand on the array `ptr` (no allocation): the
// sweep's families through k_one, the oscillatory quadratic through the
// complex sweep with the tables compiled into the library.  Returns 0, the
// HIP error code, or -1 if the launch would need more scratch than the array
// holds.
int noalloc_launch(double* ptr, int precision, int d, int K, int rule, int family, const double* params,
                   double* out, double* bound, void* stream)
{
    const bool oscq = family == SG_FAMILY_OSCILLATORY_QUADRATIC || family == SG_FAMILY_OSCILLATORY_QUADRATIC_LINEAR;
    const int G = one_workgroups(d, oscq);
    const long need = (long)kOneHead + (long)G * (oscq ? kOscqWords : kOneWords);
    if (need > (long)kNoAllocWords) return -1;
    if (oscq)
        return launch_oscq(precision, d, K, rule, G, family == SG_FAMILY_OSCILLATORY_QUADRATIC_LINEAR ? 1 : 0, nullptr,
                           nullptr, params, out, bound, ptr, stream);
    return launch_one(precision, d, K, rule, family, G, params, out, bound, ptr, stream);
}

long noalloc_capacity_words() { return (long)kNoAllocWords; }

}  // namespace sg
