// HIP kernels (gfx950) for the Smolyak dimension sweep.
//
// Method (Section 2.1 (2.6), Section 3 (3.9)-(3.11)).  With K = q - d, the
// Smolyak sum over the window equals the sum over all multi-indices of
// excess <= K of tensor products of difference rules Delta^{l_i} (the
// summation-by-coordinates form (2.9)).  For an integrand that factorises
// per coordinate after centring, f(x) = A * prod_t (1 + h_t(x_t)) with
// h_t(1/2) = 0, each tensor term factorises too, and summing over the
// multi-indices of a given excess is a coefficient of a polynomial product:
//
//   Q = A * sum_{b <= K} [z^b] prod_t delta_t(z),
//   delta_t(z) = 1 + sum_{e=1..K} Delta^{e+1}(h_t) z^e.
//
// A coordinate sweep that multiplies delta_t into a running truncated
// polynomial is the dimension iteration of Algorithm 3.3 with step 1: the
// running polynomial, indexed by the remaining level budget (the gamma
// recursion under (2.9)), is the partial function f_{t-m} of (3.11) for
// these integrands, and A is the affine partial sum (log-amplitude / phase)
// carried alongside.  Because truncated multiplication is associative and
// commutative, the sweep is split over lanes, waves and workgroups and
// merged by a deterministic tree.
//
// Per coordinate the work is: evaluate the centred factor on node pairs
// {1/2 - y, 1/2 + y} (the difference rules are symmetric, so only the even
// part s(y) = h(1/2+y) + h(1/2-y) is needed), then the within-rule sums
// delta_t[e] = sum_p dW[e][p] s_p.  Families (v = parameter * y):
//   exp-sum      h = e^{c y} - 1           s = 2(cosh v - 1)
//   oscillatory  h = e^{i a y} - 1 (Re/Im) s = 2(cos v - 1)   (the odd
//                imaginary part cancels; the phase lives in A)
//   product-peak h = D(1/2)/D(1/2+y) - 1   s = 2 y^2 (v'^2 - D(1/2) - y^2)/(D+ D-)
// all written without cancellation (Taylor series in v^2 for |v| <= 1/2).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sg_internal.hpp"

namespace sg {
namespace {

constexpr int MAXK = kMaxK;
constexpr int FAM_EXP = SG_FAMILY_EXP_SUM;
constexpr int FAM_OSC = SG_FAMILY_OSCILLATORY;
constexpr int FAM_PEAK = SG_FAMILY_PRODUCT_PEAK;

// ----------------------------------------------------------------- series
// P(z) = sum_{k>=0} 2 z^k / (2k+2)!, so that for z = v^2:
//   2 (cosh v - 1) = z P(z),   2 (cos v - 1) = -z P(-z).
// Truncation at |v| <= 1/2 (z <= 1/4): the first dropped term relative to 1
// is 2 z^8/18! < 5e-21 (FP64, 8 terms) and 2 z^4/10! < 3e-9 (FP32, 4 terms).
__device__ __forceinline__ double series64(double z)
{
    double p = 1.0 / 10461394944000.0;                 // 2/16!
    p = fma(p, z, 1.0 / 43589145600.0);                // 2/14!
    p = fma(p, z, 1.0 / 239500800.0);                  // 2/12!
    p = fma(p, z, 1.0 / 1814400.0);                    // 2/10!
    p = fma(p, z, 1.0 / 20160.0);                      // 2/8!
    p = fma(p, z, 1.0 / 360.0);                        // 2/6!
    p = fma(p, z, 1.0 / 12.0);                         // 2/4!
    p = fma(p, z, 1.0);                                // 2/2!
    return p;
}

__device__ __forceinline__ float series32(float z)
{
    float p = 1.0f / 20160.0f;
    p = fmaf(p, z, 1.0f / 360.0f);
    p = fmaf(p, z, 1.0f / 12.0f);
    p = fmaf(p, z, 1.0f);
    return p;
}

// Per-coordinate family parameters, read once per coordinate.
struct CoordParam {
    double p0;    // exp: c; osc: a; peak: beta = b^-2
    double p1;    // peak: (1 - 2u)/2
};

template <int FAM>
__device__ __forceinline__ double pair64(const CoordParam& cp, double y)
{
    if constexpr (FAM == FAM_EXP || FAM == FAM_OSC) {
        const double v = cp.p0 * y;
        const double z = v * v;
        const double av = fabs(v);
        if (av <= 0.5) return FAM == FAM_EXP ? z * series64(z) : -z * series64(-z);
        if constexpr (FAM == FAM_EXP) {
            const double E = expm1(av);            // e^v + e^-v - 2 = E^2 / (1 + E)
            return E * (E / (1.0 + E));
        } else {
            const double sn = sin(0.5 * v);        // 2(cos v - 1) = -4 sin^2(v/2)
            return -4.0 * sn * sn;
        }
    } else {
        const double beta = cp.p0, hv = cp.p1;
        const double y2 = y * y;
        const double dp = y + hv, dm = y - hv;
        const double Dp = fma(dp, dp, beta), Dm = fma(dm, dm, beta);
        // h(y) + h(-y) = 2 y^2 (3 hv^2 - beta - y^2) / (Dp Dm)
        const double num = 2.0 * y2 * (fma(3.0 * hv, hv, -beta) - y2);
        return num / (Dp * Dm);
    }
}

template <int FAM>
__device__ __forceinline__ float pair32(const CoordParam& cp, double y)
{
    if constexpr (FAM == FAM_EXP || FAM == FAM_OSC) {
        const float v = (float)(cp.p0 * y);       // one rounding of the argument
        const float z = v * v;
        const float av = fabsf(v);
        if (av <= 0.5f) return FAM == FAM_EXP ? z * series32(z) : -z * series32(-z);
        if constexpr (FAM == FAM_EXP) {
            const float E = expm1f(av);
            return E * (E / (1.0f + E));
        } else {
            const float sn = sinf(0.5f * v);
            return -4.0f * sn * sn;
        }
    } else {
        // The product-peak pair value is a rational function with no
        // transcendental; its cancellation-prone parts (y^2, the bracket and
        // the two denominators) are formed in FP64 and the value is rounded
        // once, which keeps it within half an FP32 ulp of the exact value.
        return (float)pair64<FAM_PEAK>(cp, y);
    }
}

// Compensated FP32 accumulation of w*s with w = wh + wl (two-sum on the
// running sum, exact product error by FMA, low parts gathered in lo).
__device__ __forceinline__ void acc2(float& hi, float& lo, float wh, float wl, float s)
{
    const float p = wh * s;
    const float pe = fmaf(wh, s, -p);
    const float t = hi + p;
    const float bp = t - hi;
    const float err = (hi - (t - bp)) + (p - bp);
    hi = t;
    lo = fmaf(wl, s, lo + (err + pe));
}

// ------------------------------------------------- truncated polynomials
// Monic truncated polynomials 1 + a_1 z + ... + a_K z^K; a[0] is unused.
template <int K>
__device__ __forceinline__ void pmul(double (&a)[MAXK + 1], const double (&b)[MAXK + 1])
{
#pragma unroll
    for (int k = K; k >= 1; --k) {
        double acc = a[k] + b[k];
#pragma unroll
        for (int i = 1; i < k; ++i) acc = fma(a[i], b[k - i], acc);
        a[k] = acc;
    }
}

// ------------------------------------------------ per-coordinate surplus
struct TableView {
    int np;
    const int* lb;          // level_begin
    const double* y;
    const double* dw;       // (K+1) x np
    const double* wabs;
    const float* dwh;
    const float* dwl;
};

template <int K, bool NESTED, int FAM>
__device__ __forceinline__ void surplus64(const TableView& T, const CoordParam& cp, bool want_bound,
                                          double (&del)[MAXK + 1], double& eps)
{
#pragma unroll
    for (int e = 0; e <= MAXK; ++e) del[e] = 0.0;
#pragma unroll
    for (int L = 2; L <= K + 1; ++L) {
        const int pb = T.lb[L], pe = T.lb[L + 1];
        for (int p = pb; p < pe; ++p) {
            const double s = pair64<FAM>(cp, T.y[p]);
            if (want_bound) eps = fma(T.wabs[p], fabs(s), eps);
            if constexpr (NESTED) {
#pragma unroll
                for (int e = L - 1; e <= K; ++e) del[e] = fma(T.dw[e * T.np + p], s, del[e]);
            } else {
                del[L - 1] = fma(T.dw[(L - 1) * T.np + p], s, del[L - 1]);
                if (L <= K) del[L] = fma(T.dw[L * T.np + p], s, del[L]);
            }
        }
    }
}

template <int K, bool NESTED, int FAM>
__device__ __forceinline__ void surplus32(const TableView& T, const CoordParam& cp, bool want_bound,
                                          double (&del)[MAXK + 1], double& eps)
{
    float hi[MAXK + 1], lo[MAXK + 1];
#pragma unroll
    for (int e = 0; e <= MAXK; ++e) { hi[e] = 0.0f; lo[e] = 0.0f; }
    float epsf = 0.0f;
#pragma unroll
    for (int L = 2; L <= K + 1; ++L) {
        const int pb = T.lb[L], pe = T.lb[L + 1];
        for (int p = pb; p < pe; ++p) {
            const float s = pair32<FAM>(cp, T.y[p]);
            if (want_bound) epsf = fmaf((float)T.wabs[p], fabsf(s), epsf);
            if constexpr (NESTED) {
#pragma unroll
                for (int e = L - 1; e <= K; ++e)
                    acc2(hi[e], lo[e], T.dwh[e * T.np + p], T.dwl[e * T.np + p], s);
            } else {
                acc2(hi[L - 1], lo[L - 1], T.dwh[(L - 1) * T.np + p], T.dwl[(L - 1) * T.np + p], s);
                if (L <= K) acc2(hi[L], lo[L], T.dwh[L * T.np + p], T.dwl[L * T.np + p], s);
            }
        }
    }
#pragma unroll
    for (int e = 0; e <= MAXK; ++e) del[e] = (double)hi[e] + (double)lo[e];
    eps += (double)epsf;
}

// -------------------------------------------------------- block reduction
// Merge state: running polynomial a, its absolute-value twin ab (for the
// error bound), the affine partial sum ls, sum |terms of ls|, and eps.
struct Acc {
    double a[MAXK + 1];
    double ab[MAXK + 1];
    double ls, lsabs, eps;
};

template <int K>
__device__ __forceinline__ void merge(Acc& x, const Acc& y, bool want_bound)
{
    pmul<K>(x.a, y.a);
    if (want_bound) pmul<K>(x.ab, y.ab);
    x.ls += y.ls;
    x.lsabs += y.lsabs;
    x.eps += y.eps;
}

template <int K>
__device__ __forceinline__ void shfl_acc(Acc& o, const Acc& x, int mask, bool want_bound)
{
#pragma unroll
    for (int k = 1; k <= K; ++k) o.a[k] = __shfl_xor(x.a[k], mask);
    if (want_bound) {
#pragma unroll
        for (int k = 1; k <= K; ++k) o.ab[k] = __shfl_xor(x.ab[k], mask);
    }
    o.ls = __shfl_xor(x.ls, mask);
    o.lsabs = __shfl_xor(x.lsabs, mask);
    o.eps = __shfl_xor(x.eps, mask);
}

constexpr int ACC_WORDS = 2 * MAXK + 3;   // doubles per wave in LDS

// Reduce the block's per-thread states into thread 0 (deterministic tree:
// xor butterflies inside each wave, then the wave results in wave order).
template <int K>
__device__ __forceinline__ void block_reduce(Acc& x, bool want_bound, double* smem)
{
    for (int m = 32; m >= 1; m >>= 1) {
        Acc o;
        shfl_acc<K>(o, x, m, want_bound);
        merge<K>(x, o, want_bound);
    }
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
    if (nw == 1) return;
    if (lane == 0) {
        double* s = smem + wid * ACC_WORDS;
#pragma unroll
        for (int k = 1; k <= K; ++k) { s[k - 1] = x.a[k]; s[MAXK + k - 1] = x.ab[k]; }
        s[2 * MAXK] = x.ls;
        s[2 * MAXK + 1] = x.lsabs;
        s[2 * MAXK + 2] = x.eps;
    }
    __syncthreads();
    if (wid == 0) {
        if (lane < nw) {
            const double* s = smem + lane * ACC_WORDS;
#pragma unroll
            for (int k = 1; k <= K; ++k) { x.a[k] = s[k - 1]; x.ab[k] = s[MAXK + k - 1]; }
            x.ls = s[2 * MAXK];
            x.lsabs = s[2 * MAXK + 1];
            x.eps = s[2 * MAXK + 2];
        } else {
#pragma unroll
            for (int k = 1; k <= K; ++k) { x.a[k] = 0.0; x.ab[k] = 0.0; }
            x.ls = x.lsabs = x.eps = 0.0;
        }
        for (int m = 2; m >= 1; m >>= 1) {
            Acc o;
            shfl_acc<K>(o, x, m, want_bound);
            merge<K>(x, o, want_bound);
        }
    }
}

// ------------------------------------------------------------ integrand
template <int PREC, int K, bool NESTED, int FAM>
__device__ __forceinline__ void integrand_body(const ProbDev& P, const TableDev& TD, const double* pool64,
                               const float* pool32, const double* __restrict__ params, double* out,
                               double* bound, double* smem)
{
    TableView T;
    T.np = TD.npairs;
    T.lb = TD.level_begin;
    T.y = pool64 + TD.off64;
    T.dw = T.y + T.np;
    T.wabs = T.dw + (size_t)(K + 1) * T.np;
    T.dwh = pool32 + TD.off32 + T.np;
    T.dwl = T.dwh + (size_t)(K + 1) * T.np;
    const bool want_bound = bound != nullptr;
    const int d = P.d;
    const double* prm = params + P.param_offset;

    Acc x;
#pragma unroll
    for (int k = 0; k <= MAXK; ++k) { x.a[k] = 0.0; x.ab[k] = 0.0; }
    x.ls = x.lsabs = x.eps = 0.0;

    // the sweep: each thread walks its coordinates t = tid, tid + B, ...
    for (int t = threadIdx.x; t < d; t += blockDim.x) {
        CoordParam cp;
        double lterm;
        if constexpr (FAM == FAM_EXP) {
            cp.p0 = prm[t];
            cp.p1 = 0.0;
            lterm = 0.5 * cp.p0;                      // log g_t(1/2) = c_t / 2
        } else if constexpr (FAM == FAM_OSC) {
            cp.p0 = prm[1 + t];
            cp.p1 = 0.0;
            lterm = 0.5 * cp.p0;                      // phase of g_t(1/2) = a_t / 2
        } else {
            const double b = prm[t], u = prm[d + t];
            cp.p0 = 1.0 / (b * b);
            cp.p1 = 0.5 - u;
            lterm = log(fma(cp.p1, cp.p1, cp.p0));    // log D_t(1/2) = -log g_t(1/2)
        }
        double del[MAXK + 1];
        double eps_t = 0.0;
        if constexpr (PREC == SG_PREC_FP64) surplus64<K, NESTED, FAM>(T, cp, want_bound, del, eps_t);
        else surplus32<K, NESTED, FAM>(T, cp, want_bound, del, eps_t);
        pmul<K>(x.a, del);
        if (want_bound) {
            double dab[MAXK + 1];
#pragma unroll
            for (int k = 0; k <= MAXK; ++k) dab[k] = fabs(del[k]);
            pmul<K>(x.ab, dab);
        }
        x.ls += lterm;
        x.lsabs += fabs(lterm);
        x.eps += eps_t;
    }

    block_reduce<K>(x, want_bound, smem);

    if (threadIdx.x == 0) {
        double s = 0.0, sabs = 0.0;
#pragma unroll
        for (int k = K; k >= 1; --k) { s += x.a[k]; sabs += x.ab[k]; }
        s += 1.0;
        sabs += 1.0;
        double Q, scale, amp_rel;
        const double u64 = 1.1102230246251565e-16;
        const double ls_err = u64 * (double)d * x.lsabs;   // rounding of the affine sum
        if constexpr (FAM == FAM_OSC) {
            const double phase = 2.0 * 3.141592653589793 * prm[0] + x.ls;
            const double cph = cos(phase);
            Q = cph * s;
            scale = 1.0;                                  // |cos| <= 1
            amp_rel = 0.0;
            if (want_bound) {
                const double rel = (PREC == SG_PREC_FP64 ? u64 * (4.0 + (double)T.np)
                                                         : 5.9604644775390625e-08 * 4.0);
                const double dsum = sabs * (rel * x.eps + (K + 2) * (double)(d / (int)blockDim.x + 12) * u64);
                bound[P.out_index] = dsum + fabs(s) * (ls_err + u64 * (fabs(phase) + 4.0)) + fabs(Q) * 4.0 * u64;
            }
        } else {
            const double A = exp(FAM == FAM_EXP ? x.ls : -x.ls);
            Q = A * s;
            scale = A;
            amp_rel = ls_err + 4.0 * u64 + u64 * fabs(x.ls);
            if (want_bound) {
                const double rel = (PREC == SG_PREC_FP64 ? u64 * (4.0 + (double)T.np)
                                                         : 5.9604644775390625e-08 * 4.0);
                const double dsum = sabs * (rel * x.eps + (K + 2) * (double)(d / (int)blockDim.x + 12) * u64);
                bound[P.out_index] = scale * dsum + fabs(Q) * amp_rel;
            }
        }
        out[P.out_index] = Q;
    }
}

template <int PREC, int K>
__device__ __forceinline__ void dispatch_rule_family(const ProbDev& P, const TableDev& T, const double* pool64,
                                     const float* pool32, const double* params, double* out,
                                     double* bound, double* smem)
{
    if (T.nested) {
        if (P.family == FAM_EXP) integrand_body<PREC, K, true, FAM_EXP>(P, T, pool64, pool32, params, out, bound, smem);
        else if (P.family == FAM_OSC) integrand_body<PREC, K, true, FAM_OSC>(P, T, pool64, pool32, params, out, bound, smem);
        else integrand_body<PREC, K, true, FAM_PEAK>(P, T, pool64, pool32, params, out, bound, smem);
    } else {
        if (P.family == FAM_EXP) integrand_body<PREC, K, false, FAM_EXP>(P, T, pool64, pool32, params, out, bound, smem);
        else if (P.family == FAM_OSC) integrand_body<PREC, K, false, FAM_OSC>(P, T, pool64, pool32, params, out, bound, smem);
        else integrand_body<PREC, K, false, FAM_PEAK>(P, T, pool64, pool32, params, out, bound, smem);
    }
}

// One workgroup per integrand (plan order: most expensive first).
template <int PREC>
__global__ void __launch_bounds__(256)
k_forward(const ProbDev* __restrict__ probs, const TableDev* __restrict__ tabs,
          const double* __restrict__ pool64, const float* __restrict__ pool32,
          const double* __restrict__ params, double* __restrict__ out, double* __restrict__ bound)
{
    __shared__ double smem[4 * ACC_WORDS];
    const ProbDev P = probs[blockIdx.x];
    const TableDev& T = tabs[P.table];
    switch (P.K) {
    case 0: dispatch_rule_family<PREC, 0>(P, T, pool64, pool32, params, out, bound, smem); break;
    case 1: dispatch_rule_family<PREC, 1>(P, T, pool64, pool32, params, out, bound, smem); break;
    case 2: dispatch_rule_family<PREC, 2>(P, T, pool64, pool32, params, out, bound, smem); break;
    case 3: dispatch_rule_family<PREC, 3>(P, T, pool64, pool32, params, out, bound, smem); break;
    case 4: dispatch_rule_family<PREC, 4>(P, T, pool64, pool32, params, out, bound, smem); break;
    case 5: dispatch_rule_family<PREC, 5>(P, T, pool64, pool32, params, out, bound, smem); break;
    case 6: dispatch_rule_family<PREC, 6>(P, T, pool64, pool32, params, out, bound, smem); break;
    case 7: dispatch_rule_family<PREC, 7>(P, T, pool64, pool32, params, out, bound, smem); break;
    default: dispatch_rule_family<PREC, 8>(P, T, pool64, pool32, params, out, bound, smem); break;
    }
}

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

int launch_forward(int precision, const LaunchCfg& cfg, int nprob, const ProbDev* probs,
                   const TableDev* tabs, const double* pool64, const float* pool32,
                   const double* params, double* out, double* bound, void* stream)
{
    if (nprob <= 0) return 0;
    const dim3 grid((unsigned)nprob), block((unsigned)cfg.block);
    hipStream_t s = (hipStream_t)stream;
    if (precision == SG_PREC_FP64)
        hipLaunchKernelGGL((k_forward<SG_PREC_FP64>), grid, block, 0, s, probs, tabs, pool64, pool32, params, out, bound);
    else
        hipLaunchKernelGGL((k_forward<SG_PREC_FP32_COMPENSATED>), grid, block, 0, s, probs, tabs, pool64, pool32, params, out, bound);
    return (int)hipGetLastError();
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
