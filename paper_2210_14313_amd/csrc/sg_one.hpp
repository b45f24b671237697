// One integrand of the dimension sweep split over G workgroups, with a
// deterministic ordered merge of the workgroups' partial products
// (Section 3, (3.9)-(3.11): the truncated product over coordinates is
// associative, so chunks of coordinates reduce independently and their
// partials multiply in a fixed order).
//
// Lane l of wave w of workgroup b sweeps the coordinates
// t = (4 b + w) 64 + l + j 256 G, j = 0, 1, ...; each wave reduces its lanes
// (DPP scan), the workgroup joins its four waves in wave order and writes its
// partial to scratch; the workgroup that arrives last (a counter in scratch)
// joins all G partials -- thread i takes partials i, i + 256, ... in order,
// then a fixed binary tree over the threads -- reads out the value and its
// bound, and resets the counter, so consecutive launches (and graph replays)
// need no clearing.  G = 1 skips the scratch.  The record tables of the
// table-driven path are device arrays compiled into the library, so the
// launch needs no host-built table or descriptor.
//
// Scratch layout (doubles): kOneHeadWords words whose first 32-bit word is
// the arrival counter, then G partials of ACC_WORDS doubles.
#pragma once
#include "sg_device.hpp"
#include "sg_tables_dev.inc"

namespace sg {
namespace dev {

constexpr int kOneHeadWords = 32;   // 256 bytes before the partials
constexpr int kOneTree = 256;       // threads of the final tree
static_assert(kOneHeadWords == kOneHead && ACC_WORDS == kOneWords, "scratch layout shared with the host");

// Read-out of the joined state with an explicit product-tree depth.
template <int PREC, int K, bool GAUSS>
__device__ __forceinline__ void one_readout(int rule, int family, const Acc& x, int d, const double* prm, int depth,
                                            double* out, double* bound)
{
    const int rc = rule_class_of(rule);
    constexpr int np_nested = total_pairs<RC_NESTED, K>(), np_gl2 = total_pairs<RC_GL2, K>(),
                  np_gp = total_pairs<RC_GP, K>(), np_glp = total_pairs<RC_GLP, K>();
    const int np = rc == RC_NESTED ? np_nested : rc == RC_GL2 ? np_gl2 : rc == RC_GP ? np_gp : np_glp;
    if constexpr (GAUSS) {
        if (family == FAM_GAUSS) {
            readout<PREC, K, FAM_GAUSS>(x, d, 0, prm, np, depth, out, bound);
            return;
        }
    }
    if (family == FAM_EXP) readout<PREC, K, FAM_EXP>(x, d, 0, prm, np, depth, out, bound);
    else if (family == FAM_OSC) readout<PREC, K, FAM_OSC>(x, d, 0, prm, np, depth, out, bound);
    else readout<PREC, K, FAM_PEAK>(x, d, 0, prm, np, depth, out, bound);
}

// Workgroup part: sweep, join the four waves; returns (in thread 0) the
// workgroup's partial in `x`.
template <int PREC, int K, bool GAUSS>
__device__ __forceinline__ void one_workgroup(int d, int rule, int family, int G, const double* params,
                                              double* out, double* bound, double* lds, Acc& x)
{
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    WaveInfo wi;
    wi.lw = 6;
    wi.rank = (int)blockIdx.x * 4 + w;
    wi.group = 4 * G;
    wi.nprob = 1;
    tabd::records(rule, K, &wi.r64, &wi.r32);
    wi.d = d;
    wi.out_index = 0;
    wi.param_offset = 0;
    // every wave stores its product in its LDS slot (group > 1); the bound's
    // sums are kept when a bound is asked for
    wave_dispatch_k<PREC, K, GAUSS>(rule, family, wi, params, out, bound, lds + w * ACC_WORDS);
    __syncthreads();
    if (threadIdx.x == 0) {
        Acc y;
        acc_identity<K>(x);
        acc_identity<K>(y);
        acc_load<K>(x, lds);
        for (int v = 1; v < 4; ++v) {
            acc_load<K>(y, lds + v * ACC_WORDS);
            merge<K>(x, y, true);
        }
    }
}

template <int PREC, int K, bool GAUSS>
__device__ __forceinline__ void one_body(int d, int rule, int family, int G, const double* params, double* out,
                                         double* bound, double* scratch, double* lds, int* last)
{
    Acc x;
    one_workgroup<PREC, K, GAUSS>(d, rule, family, G, params, out, bound, lds, x);
    // product-tree depth behind the result: a lane's chain, the DPP scan, the
    // join of four waves, then (G > 1) a thread's run of partials and the tree
    const int chain = (d + 256 * G - 1) / (256 * G);
    if (G == 1) {
        if (threadIdx.x == 0) one_readout<PREC, K, GAUSS>(rule, family, x, d, params, chain + 6 + 4, out, bound);
        return;
    }
    unsigned int* counter = reinterpret_cast<unsigned int*>(scratch);
    double* partials = scratch + kOneHeadWords;
    if (threadIdx.x == 0) {
        acc_store<K>(x, partials + (size_t)blockIdx.x * ACC_WORDS);
        __threadfence();
        *last = atomicAdd(counter, 1u) == (unsigned int)(G - 1);
    }
    __syncthreads();
    if (!*last) return;
    __threadfence();
    // thread i joins partials i, i + 256, ... in order, then the tree
    const int i = threadIdx.x;
    Acc a, b;
    acc_identity<K>(a);
    acc_identity<K>(b);
    for (int j = i; j < G; j += kOneTree) {
        acc_load<K>(b, partials + (size_t)j * ACC_WORDS);
        merge<K>(a, b, true);
    }
    __syncthreads();   // the workgroup's wave slots are reused below
    acc_store<K>(a, lds + i * ACC_WORDS);
    __syncthreads();
    // tree over the threads holding partials (threads at or above the next
    // power of two of min(G, kOneTree) hold the identity; skipping their
    // levels changes no bit, merging with the identity being exact)
    int top = 1;
    while (top < G && top < kOneTree) top <<= 1;
    for (int s = top >> 1; s >= 1; s >>= 1) {
        if (i < s) {
            acc_load<K>(a, lds + i * ACC_WORDS);
            acc_load<K>(b, lds + (i + s) * ACC_WORDS);
            merge<K>(a, b, true);
            acc_store<K>(a, lds + i * ACC_WORDS);
        }
        __syncthreads();
    }
    if (i == 0) {
        acc_load<K>(a, lds);
        const int depth = chain + 6 + 4 + (G + kOneTree - 1) / kOneTree + 8;
        one_readout<PREC, K, GAUSS>(rule, family, a, d, params, depth, out, bound);
        atomicExch(counter, 0u);   // ready for the next launch
    }
}

// One integrand (param_offset 0 in params), out[0] and bound[0] (bound may be
// null), G workgroups of 256 threads; scratch holds kOneHeadWords + G *
// ACC_WORDS doubles with the counter at zero (G > 1), left at zero.
template <int PREC, int KMAXP, bool GAUSS>
__global__ void __launch_bounds__(256)
k_one(int d, int K, int rule, int family, int G, const double* __restrict__ params, double* __restrict__ out,
      double* __restrict__ bound, double* __restrict__ scratch)
{
    __shared__ double lds[kOneTree * ACC_WORDS];
    __shared__ int last;
    static_for<0, KMAXP + 1>([&](auto kc) __attribute__((always_inline)) {
        if (K == decltype(kc)::value)
            one_body<PREC, decltype(kc)::value, GAUSS>(d, rule, family, G, params, out, bound, scratch, lds, &last);
    });
}

}  // namespace dev

// Launch the split sweep of one integrand (see k_one): precision mode P.
template <int P>
int launch_one_inst(int d, int K, int rule, int family, int G, const double* params, double* out, double* bound,
                    double* scratch, void* stream)
{
    hipLaunchKernelGGL((dev::k_one<P, kMaxK, true>), dim3((unsigned)G), dim3(256), 0, (hipStream_t)stream, d, K,
                       rule, family, G, params, out, bound, scratch);
    return (int)hipGetLastError();
}

}  // namespace sg
