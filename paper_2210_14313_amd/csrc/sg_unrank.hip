// Multi-index unranking kernel and the precision dispatchers of the
// forward and reverse sweeps.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sg_internal.hpp"

namespace sg {
namespace {

// ------------------------------------------------------------- unranking
// Canonical order of the window of (2.6): excess ascending, then
// (l_1..l_d) in decreasing lexicographic order.  W[n * (d+1) + parts] holds
// the number of weak compositions of n into `parts` parts (host-computed,
// exact, n <= K).  One thread per rank, one workgroup per block of ranks.
__global__ void __launch_bounds__(256)
k_unrank(int d, int q, uint64_t rank0, uint64_t count, int max_nnz, const uint64_t* __restrict__ W,
         int32_t* __restrict__ coords, int32_t* __restrict__ levels, int32_t* __restrict__ nnz)
{
    const uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= count) return;
    const int K = q - d;
    const int stride = d + 1;
    auto weak = [&](int n, int parts) -> uint64_t { return W[(size_t)n * stride + parts]; };
    uint64_t r = rank0 + g;
    int e = K - d + 1 > 0 ? K - d + 1 : 0;
    for (; e < K; ++e) {
        const uint64_t c = weak(e, d);
        if (r < c) break;
        r -= c;
    }
    int32_t* co = coords + g * max_nnz;
    int32_t* le = levels + g * max_nnz;
    for (int k = 0; k < max_nnz; ++k) { co[k] = -1; le[k] = 0; }
    int i = 0, rem = e, k = 0;
    while (rem > 0 && k < max_nnz) {
        const uint64_t total = weak(rem, d - i);
        const uint64_t T = total - r;
        int lo = i, hi = d - 1;
        while (lo < hi) {
            const int mid = lo + (hi - lo + 1) / 2;
            if (weak(rem, d - mid) >= T) lo = mid; else hi = mid - 1;
        }
        const int j = lo;
        r -= total - weak(rem, d - j);
        int a = rem;
        for (; a > 1; --a) {
            const uint64_t cnt = weak(rem - a, d - j - 1);
            if (r < cnt) break;
            r -= cnt;
        }
        co[k] = j;
        le[k] = a + 1;
        ++k;
        rem -= a;
        i = j + 1;
    }
    nnz[g] = k;
}


}  // namespace

template <int P, int KM, bool G>
int launch_forward_inst(int, const FwdWG*, unsigned int*, int, const double*, const float*, const double*, double*,
                        double*, void*);
template <int P, int KM, bool G>
int forward_capacity_inst();
int launch_adjoint_p0(bool, int, const WGDesc*, const ProbDev*, const double*, const float*, const double*,
                      const double*, double*, double*, void*);
int launch_adjoint_p1(bool, int, const WGDesc*, const ProbDev*, const double*, const float*, const double*,
                      const double*, double*, double*, void*);

// The instantiation for a precision mode and the plan's launch class: the
// smallest K class covering the plan's problems (fewer registers, more waves
// per SIMD), or, for a plan holding gaussian problems (kmax = kKmaxGauss),
// the K <= 8 kernel built with that family.
template <int P>
static int launch_forward_p(int kmax, int nwg, const FwdWG* wgs, unsigned int* queue, int qgrid, const double* pool64,
                            const float* pool32, const double* params, double* out, double* bound, void* stream)
{
    if (kmax <= 4)
        return launch_forward_inst<P, 4, false>(nwg, wgs, queue, qgrid, pool64, pool32, params, out, bound, stream);
    if (kmax <= 6)
        return launch_forward_inst<P, 6, false>(nwg, wgs, queue, qgrid, pool64, pool32, params, out, bound, stream);
    if (kmax <= kMaxK)
        return launch_forward_inst<P, 8, false>(nwg, wgs, queue, qgrid, pool64, pool32, params, out, bound, stream);
    return launch_forward_inst<P, 8, true>(nwg, wgs, queue, qgrid, pool64, pool32, params, out, bound, stream);
}

template <int P>
static int forward_capacity_p(int kmax)
{
    return kmax <= 4 ? forward_capacity_inst<P, 4, false>()
           : kmax <= 6 ? forward_capacity_inst<P, 6, false>()
           : kmax <= kMaxK ? forward_capacity_inst<P, 8, false>()
                           : forward_capacity_inst<P, 8, true>();
}

int launch_forward(int precision, int kmax, int nwg, const FwdWG* wgs, unsigned int* queue, int qgrid,
                   const double* pool64, const float* pool32, const double* params, double* out, double* bound,
                   void* stream)
{
    if (precision == SG_PREC_FP64)
        return launch_forward_p<0>(kmax, nwg, wgs, queue, qgrid, pool64, pool32, params, out, bound, stream);
    if (precision == SG_PREC_FP32_COMPENSATED)
        return launch_forward_p<1>(kmax, nwg, wgs, queue, qgrid, pool64, pool32, params, out, bound, stream);
    return launch_forward_p<2>(kmax, nwg, wgs, queue, qgrid, pool64, pool32, params, out, bound, stream);
}

int forward_capacity(int precision, int kmax)
{
    if (precision == SG_PREC_FP64) return forward_capacity_p<0>(kmax);
    if (precision == SG_PREC_FP32_COMPENSATED) return forward_capacity_p<1>(kmax);
    return forward_capacity_p<2>(kmax);
}

template <int P>
int launch_one_inst(int d, int K, int rule, int family, int G, const double* params, double* out, double* bound,
                    double* scratch, void* stream);

int launch_one(int precision, int d, int K, int rule, int family, int G, const double* params, double* out,
               double* bound, double* scratch, void* stream)
{
    if (precision == SG_PREC_FP64)
        return launch_one_inst<0>(d, K, rule, family, G, params, out, bound, scratch, stream);
    if (precision == SG_PREC_FP32_COMPENSATED)
        return launch_one_inst<1>(d, K, rule, family, G, params, out, bound, scratch, stream);
    return launch_one_inst<2>(d, K, rule, family, G, params, out, bound, scratch, stream);
}

int launch_adjoint(int precision, bool gauss, int nwg, const WGDesc* wgs, const ProbDev* probs,
                   const double* pool64, const float* pool32, const double* params, const double* gout,
                   double* grad, double* ws, void* stream)
{
    return precision == SG_PREC_FP64
               ? launch_adjoint_p0(gauss, nwg, wgs, probs, pool64, pool32, params, gout, grad, ws, stream)
               : launch_adjoint_p1(gauss, nwg, wgs, probs, pool64, pool32, params, gout, grad, ws, stream);
}

int launch_unrank(int d, int q, uint64_t rank0, uint64_t count, int max_nnz,
                  const uint64_t* W, int /*rows*/, int32_t* coords, int32_t* levels, int32_t* nnz,
                  void* stream)
{
    if (count == 0) return 0;
    const unsigned blocks = (unsigned)((count + 255) / 256);
    hipLaunchKernelGGL(k_unrank, dim3(blocks), dim3(256), 0, (hipStream_t)stream, d, q, rank0, count,
                       max_nnz, W, coords, levels, nnz);
    return (int)hipGetLastError();
}

const char* device_error_string(int code)
{
    return hipGetErrorString((hipError_t)code);
}

}  // namespace sg
