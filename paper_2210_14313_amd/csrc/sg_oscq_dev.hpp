// Factorised sweep for the oscillatory quadratic cos(2 pi w + sum_t a_t (x_t - u_t)^2),
// optionally with a linear term sum_t c_t x_t in the phase (the sines of
// (4.1)/(4.2) in any dimension): device code of the forward
// sweep, templated on the precision mode (node values in FP64, or in FP32
// with compensated FP32 or FP64 within-rule sums; truncated products, phase
// and read-out in FP64 in every mode), and the helpers the reverse sweep
// shares.
//
// Per coordinate the factor g_t(x) = e^{i (a_t (x - u_t)^2 + c_t x)}, centred
// at x = 1/2 and written in y = x - 1/2, is g_t(1/2) (1 + h_t(y)) with
// h_t(y) = e^{i (a_t y^2 + beta_t y)} - 1, beta_t = a_t (1 - 2 u_t) + c_t
// (c_t = 0 without the linear term).  The difference rules are symmetric
// about 1/2, so each sees only the even part, through the pair value
// h(y) + h(-y) = 2 (e^{i a y^2} cos(beta y) - 1): complex, unlike the linear
// oscillatory family whose pair values are real.  The surpluses delta_t[e]
// (e = 1..K) are therefore complex, and the Smolyak sum (2.6) is
// Q = Re(e^{i (2 pi w + sum_t (a_t (1/2 - u_t)^2 + c_t / 2))} sum_{b <= K} [z^b] prod_t D_t(z)),
// D_t(z) = 1 + sum_e delta_t[e] z^e, with complex truncated products.
//
// A plan gives each oscillatory-quadratic integrand one workgroup of 256
// threads; the plan-free path splits one integrand over G workgroups.  Each
// thread sweeps the coordinates t = b 256 + tid + j 256 G, a wave combines its
// lanes by an xor butterfly of complex truncated products, the first thread
// joins the four waves in wave order, and with G > 1 the workgroups' partials
// are joined in a fixed order by the last workgroup to finish (oscq_body).
#pragma once

#include "sg_device.hpp"
#include "sg_oscq.hpp"
#include "sg_tables_dev.inc"

namespace sg {
namespace dev {

constexpr int OSCQ_WORDS = 2 * MAXK + 4;   // doubles per wave in LDS
static_assert(OSCQ_WORDS == kOscqWords, "partial layout shared with the host");

// a <- a * b for monic complex truncated polynomials (coefficients 1..K).
template <int K>
__device__ __forceinline__ void cpmul(double (&ar)[MAXK + 1], double (&ai)[MAXK + 1], const double (&br)[MAXK + 1],
                                      const double (&bi)[MAXK + 1])
{
#pragma unroll
    for (int k = K; k >= 1; --k) {
        double sr = ar[k] + br[k], si = ai[k] + bi[k];
#pragma unroll
        for (int i = 1; i < k; ++i) {
            sr = fma(ar[i], br[k - i], sr);
            sr = fma(-ai[i], bi[k - i], sr);
            si = fma(ar[i], bi[k - i], si);
            si = fma(ai[i], br[k - i], si);
        }
        ar[k] = sr;
        ai[k] = si;
    }
}

// Pair value 2 (e^{i t1} cos t2 - 1), t1 = a y^2, t2 = beta y, free of
// cancellation: real part -4 (sin^2(t1/2) cos t2 + sin^2(t2/2)), imaginary
// part 4 sin(t1/2) cos(t1/2) cos t2.  `mag` bounds |re| + |im| plus the
// arguments' magnitudes, against which the bound charges each pair (the
// arguments carry a relative rounding, the sines an absolute one); t2's
// magnitude is taken as bmag |y| with bmag = |a (1 - 2u)| + |c| >= |beta|,
// which also covers the rounding of beta's two terms when they cancel.
__device__ __forceinline__ void pair_oscq(double a, double beta, double bmag, double y, double& re, double& im,
                                          double& mag)
{
    const double t1 = a * (y * y), t2 = beta * y;
    double s1, c1, s2, c2h;
    sincos(0.5 * t1, &s1, &c1);
    sincos(0.5 * t2, &s2, &c2h);
    const double c2 = fma(-2.0 * s2, s2, 1.0);
    re = -4.0 * fma(s1 * s1, c2, s2 * s2);
    im = 4.0 * (s1 * c1) * c2;
    mag = fabs(re) + fabs(im) + fabs(t1) + bmag * fabs(y);
}

// The same pair value in FP32 (the FP32 precision modes).  With
// P(t) = 2 (cos t - 1) = -t^2 (1 - t^2/12 + ...) and cos t2 = 1 + P(t2)/2 the
// real part is P(t1) cos t2 + P(t2), two terms of one sign (no cancellation
// while |t2| <= 1), and the imaginary part 2 t1 (sin t1 / t1) cos t2; both
// series are taken on |t| <= 1, where their first dropped terms lie below
// 2^-27 relative.  The arguments are formed in FP64 and rounded once.  Error
// count on the series path, in units of 2^-24 relative to each part: the
// argument 1, its square 3, a series 2, P 6, cos t2 4, real part 11,
// imaginary part 10; the bound charges 14 units of `mag` (which is rounded
// down by at most one).  Outside the series range the FP64 values are
// rounded once (their error is below one unit of `mag`).
__device__ __forceinline__ void pair_oscq32(double a, double beta, double bmag, double y, float& re, float& im,
                                            float& mag)
{
    const float t1 = (float)(a * (y * y)), t2 = (float)(beta * y);
    if (fabsf(t1) <= 1.0f && fabsf(t2) <= 1.0f) {
        const float z1 = -(t1 * t1), z2 = -(t2 * t2);
        const float p1 = z1 * series32w(z1), p2 = z2 * series32w(z2);
        const float c2 = fmaf(0.5f, p2, 1.0f);
        re = fmaf(p1, c2, p2);
        im = (2.0f * t1) * (series_s32w(z1) * c2);
        mag = fabsf(re) + fabsf(im) + fabsf(t1) + (float)(bmag * fabs(y));
        return;
    }
    double r, i, m;
    pair_oscq(a, beta, bmag, y, r, i, m);
    re = (float)r;
    im = (float)i;
    mag = (float)m;
}

// Complex surpluses of one coordinate from the (rule class, K) record table
// (per pair: y, dW[elo..ehi], sum_e |dW|); eps accumulates sum_e |dW| * mag.
template <int K, int RC>
__device__ __forceinline__ void surplus_oscq(const double* __restrict__ r64, double a, double beta, double bmag,
                                             double (&dr)[MAXK + 1], double (&di)[MAXK + 1], double& eps)
{
#pragma unroll
    for (int e = 0; e <= MAXK; ++e) { dr[e] = 0.0; di[e] = 0.0; }
    static_for<2, K + 2>([&](auto Lc) {
        constexpr int L = decltype(Lc)::value;
        constexpr int np = rc_pairs(RC, L), lo = rc_elo(L), hi = rc_ehi(RC, K, L);
        constexpr int rl = rc_rec64(RC, K, L), off = rc_off64(RC, K, L);
#pragma unroll 2
        for (int j = 0; j < np; ++j) {
            const double* r = r64 + off + j * rl;
            double pr, pi, pm;
            pair_oscq(a, beta, bmag, r[0], pr, pi, pm);
#pragma unroll
            for (int e = lo; e <= hi; ++e) {
                dr[e] = fma(r[1 + e - lo], pr, dr[e]);
                di[e] = fma(r[1 + e - lo], pi, di[e]);
            }
            eps = fma(r[rl - 1], pm, eps);
        }
    });
}

// Complex surpluses with FP32 node values: PREC = SG_PREC_FP32_COMPENSATED
// sums each part with the two-sum compensated FP32 accumulation against the
// FP32 hi + lo weights (r32 records), SG_PREC_FP32_FP64_SUM in FP64 against
// the FP64 weights; eps as in surplus_oscq.
template <int PREC, int K, int RC>
__device__ __forceinline__ void surplus_oscq32(const double* __restrict__ r64, const float* __restrict__ r32,
                                               double a, double beta, double bmag, double (&dr)[MAXK + 1],
                                               double (&di)[MAXK + 1], double& eps)
{
    float rh[MAXK + 1], rlo[MAXK + 1], ih[MAXK + 1], ilo[MAXK + 1];
#pragma unroll
    for (int e = 0; e <= MAXK; ++e) {
        dr[e] = 0.0;
        di[e] = 0.0;
        rh[e] = rlo[e] = ih[e] = ilo[e] = 0.0f;
    }
    static_for<2, K + 2>([&](auto Lc) {
        constexpr int L = decltype(Lc)::value;
        constexpr int np = rc_pairs(RC, L), lo = rc_elo(L), hi = rc_ehi(RC, K, L);
        constexpr int rl = rc_rec64(RC, K, L), off = rc_off64(RC, K, L);
        constexpr int rl32 = rc_rec32(RC, K, L), off32 = rc_off32(RC, K, L);
#pragma unroll 2
        for (int j = 0; j < np; ++j) {
            const double* r = r64 + off + j * rl;
            float pr, pi, pm;
            pair_oscq32(a, beta, bmag, r[0], pr, pi, pm);
            if constexpr (PREC == SG_PREC_FP32_COMPENSATED) {
                const float* w = r32 + off32 + j * rl32;
#pragma unroll
                for (int e = lo; e <= hi; ++e) {
                    acc2(rh[e], rlo[e], w[2 * (e - lo)], w[2 * (e - lo) + 1], pr);
                    acc2(ih[e], ilo[e], w[2 * (e - lo)], w[2 * (e - lo) + 1], pi);
                }
            } else {
#pragma unroll
                for (int e = lo; e <= hi; ++e) {
                    dr[e] = fma(r[1 + e - lo], (double)pr, dr[e]);
                    di[e] = fma(r[1 + e - lo], (double)pi, di[e]);
                }
            }
            eps = fma(r[rl - 1], (double)pm, eps);
        }
    });
    if constexpr (PREC == SG_PREC_FP32_COMPENSATED) {
#pragma unroll
        for (int e = 0; e <= MAXK; ++e) {
            dr[e] = (double)rh[e] + (double)rlo[e];
            di[e] = (double)ih[e] + (double)ilo[e];
        }
    }
}

// State of a partial complex sweep: the truncated product (real and
// imaginary coefficients 1..K) and the sums the read-out and bound need.
struct OscqAcc {
    double ar[MAXK + 1], ai[MAXK + 1];
    double m, eps, ph, phabs;
};

template <int K>
__device__ __forceinline__ void oscq_identity(OscqAcc& x)
{
#pragma unroll
    for (int k = 0; k <= MAXK; ++k) { x.ar[k] = 0.0; x.ai[k] = 0.0; }
    x.m = x.eps = x.ph = x.phabs = 0.0;
}

template <int K>
__device__ __forceinline__ void oscq_merge(OscqAcc& x, const OscqAcc& y)
{
    cpmul<K>(x.ar, x.ai, y.ar, y.ai);
    x.m += y.m;
    x.eps += y.eps;
    x.ph += y.ph;
    x.phabs += y.phabs;
}

template <int K>
__device__ __forceinline__ void oscq_store(const OscqAcc& x, double* s)
{
#pragma unroll
    for (int k = 1; k <= K; ++k) {
        s[k - 1] = x.ar[k];
        s[MAXK + k - 1] = x.ai[k];
    }
    s[2 * MAXK] = x.m;
    s[2 * MAXK + 1] = x.eps;
    s[2 * MAXK + 2] = x.ph;
    s[2 * MAXK + 3] = x.phabs;
}

template <int K>
__device__ __forceinline__ void oscq_load(OscqAcc& x, const double* s)
{
#pragma unroll
    for (int k = 1; k <= K; ++k) {
        x.ar[k] = s[k - 1];
        x.ai[k] = s[MAXK + k - 1];
    }
    x.m = s[2 * MAXK];
    x.eps = s[2 * MAXK + 1];
    x.ph = s[2 * MAXK + 2];
    x.phabs = s[2 * MAXK + 3];
}

// Partial sweep of workgroup b of G over the coordinates
// t = b 256 + tid + j 256 G; thread 0 returns the workgroup's state (its
// four waves joined in wave order).
template <int PREC, int K, int RC>
__device__ void oscq_partial(int d, int b, int G, bool lin, const double* __restrict__ r64,
                             const float* __restrict__ r32, const double* __restrict__ prm, double* lds, OscqAcc& x)
{
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    oscq_identity<K>(x);
    for (int t = b * 256 + tid; t < d; t += 256 * G) {
        const double a = prm[1 + t], hv = 0.5 - prm[1 + d + t];
        const double c = lin ? prm[1 + 2 * d + t] : 0.0;
        const double ab = a * (2.0 * hv);
        const double beta = ab + c, bmag = fabs(ab) + fabs(c);
        double dr[MAXK + 1], di[MAXK + 1], e_t = 0.0;
        int opaque = 0;
        asm volatile("" : "+s"(opaque));
        if constexpr (PREC == SG_PREC_FP64) surplus_oscq<K, RC>(r64 + opaque, a, beta, bmag, dr, di, e_t);
        else surplus_oscq32<PREC, K, RC>(r64 + opaque, r32 + opaque, a, beta, bmag, dr, di, e_t);
        cpmul<K>(x.ar, x.ai, dr, di);
        double mt = 0.0;
#pragma unroll
        for (int k = 1; k <= K; ++k) mt += fabs(dr[k]) + fabs(di[k]);
        x.m += mt;
        x.eps += e_t;
        const double sq = a * (hv * hv);
        x.ph += fma(0.5, c, sq);                     // phase of g_t(1/2)
        x.phabs += fabs(sq) + fabs(0.5 * c);
    }
    for (int off = 32; off >= 1; off >>= 1) {
        OscqAcc y;
#pragma unroll
        for (int k = 1; k <= K; ++k) {
            y.ar[k] = __shfl_xor(x.ar[k], off);
            y.ai[k] = __shfl_xor(x.ai[k], off);
        }
        y.m = __shfl_xor(x.m, off);
        y.eps = __shfl_xor(x.eps, off);
        y.ph = __shfl_xor(x.ph, off);
        y.phabs = __shfl_xor(x.phabs, off);
        oscq_merge<K>(x, y);
    }
    if (lane == 0) oscq_store<K>(x, lds + w * OSCQ_WORDS);
    __syncthreads();
    if (tid != 0) return;
    for (int v = 1; v < 4; ++v) {
        OscqAcc y;
        oscq_load<K>(y, lds + v * OSCQ_WORDS);
        oscq_merge<K>(x, y);
    }
}

// Q = Re(e^{i (2 pi w + ph)} S) and its bound; depth: levels of the product
// tree behind the joined state.
template <int PREC, int K, int RC>
__device__ void oscq_readout(const OscqAcc& x, int d, int depth, const double* __restrict__ prm,
                             double* __restrict__ out, double* __restrict__ bound)
{
    double sr = 0.0, si = 0.0;
#pragma unroll
    for (int k = K; k >= 1; --k) {
        sr += x.ar[k];
        si += x.ai[k];
    }
    sr += 1.0;
    const double wp = 2.0 * 3.141592653589793 * prm[0];
    const double phase = wp + x.ph;
    double sn, cs;
    sincos(phase, &sn, &cs);
    const double Q = fma(cs, sr, -sn * si);
    out[0] = Q;
    if (bound) {
        const double u64 = 1.1102230246251565e-16;
        // coefficients of every partial product are bounded in sum by
        // T_K(m), m = sum_t sum_e (|Re delta_t[e]| + |Im delta_t[e]|) (as for
        // the real sweep, moduli in place of absolute values); m's FP64 sum
        // of non-negative terms, at most d + depth roundings, raised first
        const double m_up = x.m * (1.0 + (double)(2 * (d + depth + 4)) * u64);
        const double sabs = abs_product_bound<K>(m_up);
        // per pair term, relative to mag: FP64 values 12 roundings and one
        // FMA chain over the table's pairs; FP32 values 14 units of 2^-24
        // (pair_oscq32) plus, with compensated FP32 sums, one rounding of
        // the product and the second-order 2^-47 per pair of the low-part
        // chain, or, with FP64 sums, the FP64 chain
        const double np = (double)total_pairs<RC, K>();
        const double u32 = 5.9604644775390625e-08;
        const double rel = PREC == SG_PREC_FP64               ? u64 * (12.0 + np)
                           : PREC == SG_PREC_FP32_COMPENSATED ? u32 * 16.0 + 7.105427357601002e-15 * np
                                                              : u32 * 15.0 + u64 * (8.0 + np);
        // product tree: a complex truncated product rounds each component at
        // most 2K + 2 times per level
        const double dsum = sabs * (rel * x.eps + (2.0 * K + 4.0) * (double)depth * u64);
        // phase: d - 1 additions of terms rounded at most three times each,
        // and 2 pi w
        const double ph_err = u64 * (double)(d + 4) * x.phabs + 2.0 * u64 * fabs(wp);
        const double smag = sqrt(fma(sr, sr, si * si)) + dsum;
        bound[0] = dsum + smag * (ph_err + u64 * (fabs(phase) + 8.0));
    }
}

// One integrand on G workgroups: G = 1 reads out directly; otherwise each
// workgroup writes its partial to scratch (after kOscqHeadWords words whose
// first 32-bit word is the arrival counter), and the last to arrive joins
// the G partials (thread i those i, i + 256, ... in order, then a fixed tree
// over the threads), reads out, and resets the counter.
constexpr int kOscqHeadWords = 32;
static_assert(kOscqHeadWords == kOscqScratchHead, "scratch layout shared with the host");

template <int PREC, int K, int RC>
__device__ void oscq_body(int d, int b, int G, bool lin, const double* __restrict__ r64,
                          const float* __restrict__ r32, const double* __restrict__ prm, double* __restrict__ out,
                          double* __restrict__ bound, double* __restrict__ scratch, double* lds, int* last)
{
    OscqAcc x;
    oscq_partial<PREC, K, RC>(d, b, G, lin, r64, r32, prm, lds, x);
    // a thread's ceil(d / (256 G)) coordinates, 6 butterfly levels, 3 wave joins
    const int chain = (d + 256 * G - 1) / (256 * G);
    if (G == 1) {
        if (threadIdx.x == 0) oscq_readout<PREC, K, RC>(x, d, chain + 9, prm, out, bound);
        return;
    }
    unsigned int* counter = reinterpret_cast<unsigned int*>(scratch);
    double* partials = scratch + kOscqHeadWords;
    if (threadIdx.x == 0) {
        oscq_store<K>(x, partials + (size_t)b * OSCQ_WORDS);
        __threadfence();
        *last = atomicAdd(counter, 1u) == (unsigned int)(G - 1);
    }
    __syncthreads();
    if (!*last) return;
    __threadfence();
    const int i = threadIdx.x;
    OscqAcc a, c;
    oscq_identity<K>(a);
    for (int j = i; j < G; j += 256) {
        oscq_load<K>(c, partials + (size_t)j * OSCQ_WORDS);
        oscq_merge<K>(a, c);
    }
    __syncthreads();
    oscq_store<K>(a, lds + i * OSCQ_WORDS);
    __syncthreads();
    // tree over the threads holding partials (threads at or above the next
    // power of two of min(G, 256) hold the identity; skipping their levels
    // changes no bit, merging with the identity being exact)
    int top = 1;
    while (top < G && top < 256) top <<= 1;
    for (int s = top >> 1; s >= 1; s >>= 1) {
        if (i < s) {
            oscq_load<K>(a, lds + i * OSCQ_WORDS);
            oscq_load<K>(c, lds + (i + s) * OSCQ_WORDS);
            oscq_merge<K>(a, c);
            oscq_store<K>(a, lds + i * OSCQ_WORDS);
        }
        __syncthreads();
    }
    if (i == 0) {
        oscq_load<K>(a, lds);
        oscq_readout<PREC, K, RC>(a, d, chain + 9 + (G + 255) / 256 + 8, prm, out, bound);
        atomicExch(counter, 0u);
    }
}

// b: this workgroup's index among the G of one integrand; lin: the
// parameters carry the linear coefficients c[d] after u[d].
template <int PREC>
__device__ __forceinline__ void oscq_dispatch(int d, int K, int rule, int b, int G, bool lin, const double* r64,
                                              const float* r32, const double* prm, double* out, double* bound,
                                              double* scratch, double* lds, int* last)
{
    const int rc = rule_class_of(rule);
    switch_k<MAXK>(K, [&](auto kc) {
        constexpr int KK = decltype(kc)::value;
        if (rc == RC_NESTED)
            oscq_body<PREC, KK, RC_NESTED>(d, b, G, lin, r64, r32, prm, out, bound, scratch, lds, last);
        else if (rc == RC_GL2)
            oscq_body<PREC, KK, RC_GL2>(d, b, G, lin, r64, r32, prm, out, bound, scratch, lds, last);
        else if (rc == RC_GP)
            oscq_body<PREC, KK, RC_GP>(d, b, G, lin, r64, r32, prm, out, bound, scratch, lds, last);
        else
            oscq_body<PREC, KK, RC_GLP>(d, b, G, lin, r64, r32, prm, out, bound, scratch, lds, last);
    });
}

// One integrand on G workgroups (scratch: see oscq_body; unused for G = 1).
// pool64 == nullptr: the (rule, K) records compiled into the library.
template <int PREC>
__global__ void __launch_bounds__(256)
k_oscq(int d, int K, int rule, int G, int lin, const double* __restrict__ pool64, const float* __restrict__ pool32,
       const double* __restrict__ params, double* __restrict__ out, double* __restrict__ bound,
       double* __restrict__ scratch)
{
    __shared__ double lds[256 * OSCQ_WORDS];
    __shared__ int last;
    const double* r64 = pool64;
    const float* r32 = pool32;
    if (!r64) tabd::records(rule, K, &r64, &r32);
    oscq_dispatch<PREC>(d, K, rule, (int)blockIdx.x, G, lin != 0, r64, r32, params, out, bound, scratch, lds, &last);
}

// Workgroup b runs descriptor b (one workgroup per integrand).
template <int PREC>
__global__ void __launch_bounds__(256)
k_oscq_batch(const OscqDesc* __restrict__ descs, const double* __restrict__ pool64, const float* __restrict__ pool32,
             const double* __restrict__ params, double* __restrict__ out, double* __restrict__ bound)
{
    __shared__ double lds[4 * OSCQ_WORDS];
    __shared__ int last;
    const OscqDesc q = descs[blockIdx.x];
    oscq_dispatch<PREC>(q.d, q.K, q.rule, 0, 1, q.lin != 0, pool64 + q.off64, pool32 + q.off32,
                        params + q.param_offset, out + q.out_index, bound ? bound + q.out_index : nullptr, nullptr,
                        lds, &last);
}

}  // namespace dev

// Launchers of one precision mode (instantiated in sg_oscq.hip for FP64 and
// in sg_oscq_p1.hip / sg_oscq_p2.hip for the FP32 modes).
template <int PREC>
int launch_oscq_prec(int d, int K, int rule, int G, int lin, const double* pool64, const float* pool32,
                     const double* params, double* out, double* bound, double* scratch, void* stream)
{
    hipLaunchKernelGGL(dev::k_oscq<PREC>, dim3((unsigned)G), dim3(256), 0, (hipStream_t)stream, d, K, rule, G, lin,
                       pool64, pool32, params, out, bound, scratch);
    return (int)hipGetLastError();
}

template <int PREC>
int launch_oscq_batch_prec(int n, const OscqDesc* descs, const double* pool64, const float* pool32,
                           const double* params, double* out, double* bound, void* stream)
{
    if (n <= 0) return 0;
    hipLaunchKernelGGL(dev::k_oscq_batch<PREC>, dim3((unsigned)n), dim3(256), 0, (hipStream_t)stream, descs, pool64,
                       pool32, params, out, bound);
    return (int)hipGetLastError();
}

}  // namespace sg
