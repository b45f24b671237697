// Factorised sweep for the oscillatory quadratic cos(2 pi w + sum_t a_t (x_t - u_t)^2)
// (the sines of (4.1)/(4.2) in any dimension), FP64.
//
// Per coordinate the factor g_t(x) = e^{i a_t (x - u_t)^2}, centred at x = 1/2
// and written in y = x - 1/2, is g_t(1/2) (1 + h_t(y)) with
// h_t(y) = e^{i a_t (y^2 + b_t y)} - 1, b_t = 1 - 2 u_t.  The difference rules
// are symmetric about 1/2, so each sees only the even part, through the pair
// value h(y) + h(-y) = 2 (e^{i a y^2} cos(a b y) - 1): complex, unlike the
// linear oscillatory family whose pair values are real.  The surpluses
// delta_t[e] (e = 1..K) are therefore complex, and the Smolyak sum (2.6) is
// Q = Re(e^{i (2 pi w + sum_t a_t (1/2 - u_t)^2)} sum_{b <= K} [z^b] prod_t D_t(z)),
// D_t(z) = 1 + sum_e delta_t[e] z^e, with complex truncated products.
//
// A plan gives each oscillatory-quadratic integrand one workgroup of 256
// threads; the plan-free path splits one integrand over G workgroups.  Each
// thread sweeps the coordinates t = b 256 + tid + j 256 G, a wave combines its
// lanes by an xor butterfly of complex truncated products, the first thread
// joins the four waves in wave order, and with G > 1 the workgroups' partials
// are joined in a fixed order by the last workgroup to finish (oscq_body).
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

// Pair value 2 (e^{i t1} cos t2 - 1), t1 = a y^2, t2 = a b y, free of
// cancellation: real part -4 (sin^2(t1/2) cos t2 + sin^2(t2/2)), imaginary
// part 4 sin(t1/2) cos(t1/2) cos t2.  `mag` bounds |re| + |im| plus the
// arguments' magnitudes, against which the bound charges each pair (the
// arguments carry a relative rounding, the sines an absolute one).
__device__ __forceinline__ void pair_oscq(double a, double b, double y, double& re, double& im, double& mag)
{
    const double t1 = a * (y * y), t2 = a * (b * y);
    double s1, c1, s2, c2h;
    sincos(0.5 * t1, &s1, &c1);
    sincos(0.5 * t2, &s2, &c2h);
    const double c2 = fma(-2.0 * s2, s2, 1.0);
    re = -4.0 * fma(s1 * s1, c2, s2 * s2);
    im = 4.0 * (s1 * c1) * c2;
    mag = fabs(re) + fabs(im) + fabs(t1) + fabs(t2);
}

// Complex surpluses of one coordinate from the (rule class, K) record table
// (per pair: y, dW[elo..ehi], sum_e |dW|); eps accumulates sum_e |dW| * mag.
template <int K, int RC>
__device__ __forceinline__ void surplus_oscq(const double* __restrict__ r64, double a, double b,
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
            pair_oscq(a, b, r[0], pr, pi, pm);
#pragma unroll
            for (int e = lo; e <= hi; ++e) {
                dr[e] = fma(r[1 + e - lo], pr, dr[e]);
                di[e] = fma(r[1 + e - lo], pi, di[e]);
            }
            eps = fma(r[rl - 1], pm, eps);
        }
    });
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
template <int K, int RC>
__device__ void oscq_partial(int d, int b, int G, const double* __restrict__ r64, const double* __restrict__ prm,
                             double* lds, OscqAcc& x)
{
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    oscq_identity<K>(x);
    for (int t = b * 256 + tid; t < d; t += 256 * G) {
        const double a = prm[1 + t], hv = 0.5 - prm[1 + d + t];
        double dr[MAXK + 1], di[MAXK + 1], e_t = 0.0;
        int opaque = 0;
        asm volatile("" : "+s"(opaque));
        surplus_oscq<K, RC>(r64 + opaque, a, 2.0 * hv, dr, di, e_t);
        cpmul<K>(x.ar, x.ai, dr, di);
        double mt = 0.0;
#pragma unroll
        for (int k = 1; k <= K; ++k) mt += fabs(dr[k]) + fabs(di[k]);
        x.m += mt;
        x.eps += e_t;
        const double term = a * (hv * hv);          // phase of g_t(1/2)
        x.ph += term;
        x.phabs += fabs(term);
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
template <int K, int RC>
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
        // exp(sum_t sum_e |delta_t[e]|) (as for the real sweep)
        const double sabs = exp(x.m) * (1.0 + 1e-13);
        // pair values: 8 roundings relative to mag; within-rule sums: one
        // FMA chain over the table's pairs
        const double rel = u64 * (8.0 + (double)total_pairs<RC, K>());
        // product tree: a complex truncated product rounds each component at
        // most 2K + 2 times per level
        const double dsum = sabs * (rel * x.eps + (2.0 * K + 4.0) * (double)depth * u64);
        // phase: d - 1 additions of terms rounded twice each, and 2 pi w
        const double ph_err = u64 * (double)(d + 3) * x.phabs + 2.0 * u64 * fabs(wp);
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

template <int K, int RC>
__device__ void oscq_body(int d, int b, int G, const double* __restrict__ r64, const double* __restrict__ prm,
                          double* __restrict__ out, double* __restrict__ bound, double* __restrict__ scratch,
                          double* lds, int* last)
{
    OscqAcc x;
    oscq_partial<K, RC>(d, b, G, r64, prm, lds, x);
    // a thread's ceil(d / (256 G)) coordinates, 6 butterfly levels, 3 wave joins
    const int chain = (d + 256 * G - 1) / (256 * G);
    if (G == 1) {
        if (threadIdx.x == 0) oscq_readout<K, RC>(x, d, chain + 9, prm, out, bound);
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
    for (int s = 128; s >= 1; s >>= 1) {
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
        oscq_readout<K, RC>(a, d, chain + 9 + (G + 255) / 256 + 8, prm, out, bound);
        atomicExch(counter, 0u);
    }
}

// b: this workgroup's index among the G of one integrand.
__device__ __forceinline__ void oscq_dispatch(int d, int K, int rule, int b, int G, const double* r64,
                                              const double* prm, double* out, double* bound, double* scratch,
                                              double* lds, int* last)
{
    const int rc = rule_class_of(rule);
    switch_k<MAXK>(K, [&](auto kc) {
        constexpr int KK = decltype(kc)::value;
        if (rc == RC_NESTED) oscq_body<KK, RC_NESTED>(d, b, G, r64, prm, out, bound, scratch, lds, last);
        else if (rc == RC_GL2) oscq_body<KK, RC_GL2>(d, b, G, r64, prm, out, bound, scratch, lds, last);
        else if (rc == RC_GP) oscq_body<KK, RC_GP>(d, b, G, r64, prm, out, bound, scratch, lds, last);
        else oscq_body<KK, RC_GLP>(d, b, G, r64, prm, out, bound, scratch, lds, last);
    });
}

// One integrand on G workgroups (scratch: see oscq_body; unused for G = 1).
// pool64 == nullptr: the (rule, K) records compiled into the library.
__global__ void __launch_bounds__(256)
k_oscq(int d, int K, int rule, int G, const double* __restrict__ pool64, const double* __restrict__ params,
       double* __restrict__ out, double* __restrict__ bound, double* __restrict__ scratch)
{
    __shared__ double lds[256 * OSCQ_WORDS];
    __shared__ int last;
    const double* r64 = pool64;
    if (!r64) {
        const float* r32;
        tabd::records(rule, K, &r64, &r32);
    }
    oscq_dispatch(d, K, rule, (int)blockIdx.x, G, r64, params, out, bound, scratch, lds, &last);
}

// Workgroup b runs descriptor b (one workgroup per integrand).
__global__ void __launch_bounds__(256)
k_oscq_batch(const OscqDesc* __restrict__ descs, const double* __restrict__ pool64,
             const double* __restrict__ params, double* __restrict__ out, double* __restrict__ bound)
{
    __shared__ double lds[4 * OSCQ_WORDS];
    __shared__ int last;
    const OscqDesc q = descs[blockIdx.x];
    oscq_dispatch(q.d, q.K, q.rule, 0, 1, pool64 + q.off64, params + q.param_offset, out + q.out_index,
                  bound ? bound + q.out_index : nullptr, nullptr, lds, &last);
}

// ------------------------------------------------------------ reverse sweep
// Gradient of Q = Re(E S), E = e^{i Phi}, Phi = 2 pi w + sum_t a_t hv_t^2
// (hv = 1/2 - u), S = sum_{b <= K} [z^b] prod_t D_t(z):
//   dQ/dw = -2 pi Im(E S);
//   dQ/dp_t = Re(E (i dPhi/dp_t S + sum_e G_t[e] d delta_t[e]/dp_t)),
// with G_t[e] = sum_{j <= K-e} [z^j] R_t and R_t = prod_{t' != t} D_t' from
// exclusive prefix and suffix products (no division), dPhi/da_t = hv_t^2,
// dPhi/du_t = -2 a_t hv_t, and per pair (t1 = a y^2, t2 = a b y, b = 2 hv)
//   d pair/da = 2 e^{i t1} (i y^2 cos t2 - b y sin t2),
//   d pair/du = 4 a y e^{i t1} sin t2.

// Derivative surpluses of one coordinate with respect to a and u.
template <int K, int RC>
__device__ __forceinline__ void dsurplus_oscq(const double* __restrict__ r64, double a, double b,
                                              double (&ar)[MAXK + 1], double (&ai)[MAXK + 1],
                                              double (&ur)[MAXK + 1], double (&ui)[MAXK + 1])
{
#pragma unroll
    for (int e = 0; e <= MAXK; ++e) { ar[e] = 0.0; ai[e] = 0.0; ur[e] = 0.0; ui[e] = 0.0; }
    static_for<2, K + 2>([&](auto Lc) {
        constexpr int L = decltype(Lc)::value;
        constexpr int np = rc_pairs(RC, L), lo = rc_elo(L), hi = rc_ehi(RC, K, L);
        constexpr int rl = rc_rec64(RC, K, L), off = rc_off64(RC, K, L);
#pragma unroll 2
        for (int j = 0; j < np; ++j) {
            const double* r = r64 + off + j * rl;
            const double y = r[0];
            double s1, c1, s2, c2;
            sincos(a * (y * y), &s1, &c1);
            sincos(a * (b * y), &s2, &c2);
            const double pr = -b * y * s2, pi = y * y * c2;     // i y^2 cos t2 - b y sin t2
            const double dar = 2.0 * (c1 * pr - s1 * pi), dai = 2.0 * (c1 * pi + s1 * pr);
            const double f = 4.0 * a * y * s2;
            const double dur = f * c1, dui = f * s1;
#pragma unroll
            for (int e = lo; e <= hi; ++e) {
                const double w = r[1 + e - lo];
                ar[e] = fma(w, dar, ar[e]);
                ai[e] = fma(w, dai, ai[e]);
                ur[e] = fma(w, dur, ur[e]);
                ui[e] = fma(w, dui, ui[e]);
            }
        }
    });
}

// Inclusive product scan of complex truncated polynomials over a wave (DPP
// steps as in the real reverse sweep).
template <int K, int CTRL, int ROW_MASK>
__device__ __forceinline__ void cpoly_dpp_step(double (&ar)[MAXK + 1], double (&ai)[MAXK + 1])
{
    double orr[MAXK + 1], oi[MAXK + 1];
    orr[0] = 0.0;
    oi[0] = 0.0;
#pragma unroll
    for (int k = 1; k <= K; ++k) {
        orr[k] = dpp_f64<CTRL, ROW_MASK>(ar[k], 0.0);
        oi[k] = dpp_f64<CTRL, ROW_MASK>(ai[k], 0.0);
    }
    cpmul<K>(ar, ai, orr, oi);
}

template <int K>
__device__ __forceinline__ void cpoly_scan_incl(double (&ar)[MAXK + 1], double (&ai)[MAXK + 1])
{
    cpoly_dpp_step<K, 0x111, 0xF>(ar, ai);
    cpoly_dpp_step<K, 0x112, 0xF>(ar, ai);
    cpoly_dpp_step<K, 0x114, 0xF>(ar, ai);
    cpoly_dpp_step<K, 0x118, 0xF>(ar, ai);
    cpoly_dpp_step<K, 0x142, 0xA>(ar, ai);
    cpoly_dpp_step<K, 0x143, 0xC>(ar, ai);
}

__device__ __forceinline__ double lane63(double v)
{
    const long long bits = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)bits, 63), hi = __builtin_amdgcn_readlane((int)(bits >> 32), 63);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

constexpr int OSCQ_GWORDS = 2 * MAXK + 2;   // doubles per wave in LDS: wave product and phase sum

// One integrand on one workgroup of 256 threads: thread i sweeps the
// coordinates t = i + 256 j.
template <int K, int RC>
__device__ void oscq_grad_body(const OscqDesc& q, const double* __restrict__ r64, const double* __restrict__ prm,
                               double g, double* __restrict__ grad, double* __restrict__ ws, double* lds)
{
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int d = q.d;
    const bool single = d <= 256;
    double* __restrict__ wsp = ws + q.ws_off;

    // pass 1: surpluses (kept in registers, or in the workspace when a
    // thread holds several coordinates), the thread's product and phase
    double Lr[MAXK + 1], Li[MAXK + 1], own_r[MAXK + 1], own_i[MAXK + 1];
#pragma unroll
    for (int k = 0; k <= MAXK; ++k) { Lr[k] = 0.0; Li[k] = 0.0; own_r[k] = 0.0; own_i[k] = 0.0; }
    double ph = 0.0;
    for (int t = tid; t < d; t += 256) {
        const double a = prm[1 + t], hv = 0.5 - prm[1 + d + t];
        double dr[MAXK + 1], di[MAXK + 1], e_t = 0.0;
        int opaque = 0;
        asm volatile("" : "+s"(opaque));
        surplus_oscq<K, RC>(r64 + opaque, a, 2.0 * hv, dr, di, e_t);
        if (single) {
#pragma unroll
            for (int k = 1; k <= K; ++k) { own_r[k] = dr[k]; own_i[k] = di[k]; }
        } else {
#pragma unroll
            for (int k = 1; k <= K; ++k) {
                wsp[(size_t)t * 2 * K + 2 * (k - 1)] = dr[k];
                wsp[(size_t)t * 2 * K + 2 * (k - 1) + 1] = di[k];
            }
        }
        cpmul<K>(Lr, Li, dr, di);
        ph += a * (hv * hv);
    }

    // exclusive prefix and suffix products over the 256 threads: DPP scans in
    // each wave (the suffix as the scan of the reversed lanes), then the
    // waves' products in wave order
    double pr[MAXK + 1], pi[MAXK + 1], sr[MAXK + 1], si[MAXK + 1];
#pragma unroll
    for (int k = 0; k <= MAXK; ++k) {
        pr[k] = Lr[k];
        pi[k] = Li[k];
        sr[k] = 0.0;
        si[k] = 0.0;
    }
#pragma unroll
    for (int k = 1; k <= K; ++k) {
        sr[k] = lane_double(Lr[k], 63 - lane);
        si[k] = lane_double(Li[k], 63 - lane);
    }
    cpoly_scan_incl<K>(pr, pi);
    cpoly_scan_incl<K>(sr, si);
    const double ph_w = wave_sum64(ph);
    // the wave's product, read from lane 63 by every lane (a cross-lane read
    // inside a one-lane branch could see values computed only for that lane)
    double tot_r[MAXK + 1], tot_i[MAXK + 1];
#pragma unroll
    for (int k = 1; k <= K; ++k) {
        tot_r[k] = lane63(pr[k]);
        tot_i[k] = lane63(pi[k]);
    }
    if (lane == 0) {
#pragma unroll
        for (int k = 1; k <= K; ++k) {
            lds[w * OSCQ_GWORDS + k - 1] = tot_r[k];
            lds[w * OSCQ_GWORDS + MAXK + k - 1] = tot_i[k];
        }
        lds[w * OSCQ_GWORDS + 2 * MAXK] = ph_w;
    }
    {
        double tr[MAXK + 1], ti[MAXK + 1];
#pragma unroll
        for (int k = 1; k <= K; ++k) {
            tr[k] = dpp_f64<0x138, 0xF>(pr[k], 0.0);     // wave_shr:1, lane 0 gets the identity
            ti[k] = dpp_f64<0x138, 0xF>(pi[k], 0.0);
            sr[k] = lane_double(sr[k], lane == 63 ? 0 : 62 - lane);
            si[k] = lane_double(si[k], lane == 63 ? 0 : 62 - lane);
        }
#pragma unroll
        for (int k = 1; k <= K; ++k) {
            pr[k] = tr[k];
            pi[k] = ti[k];
            if (lane == 63) { sr[k] = 0.0; si[k] = 0.0; }
        }
    }
    __syncthreads();
    double Sr[MAXK + 1], Si[MAXK + 1], wpr[MAXK + 1], wpi[MAXK + 1], wsr[MAXK + 1], wsi[MAXK + 1];
#pragma unroll
    for (int k = 0; k <= MAXK; ++k) { Sr[k] = 0.0; Si[k] = 0.0; wpr[k] = 0.0; wpi[k] = 0.0; wsr[k] = 0.0; wsi[k] = 0.0; }
    double phase = 2.0 * 3.141592653589793 * prm[0];
    for (int v = 0; v < 4; ++v) {
        double orr[MAXK + 1], oi[MAXK + 1];
        orr[0] = 0.0;
        oi[0] = 0.0;
#pragma unroll
        for (int k = 1; k <= K; ++k) {
            orr[k] = lds[v * OSCQ_GWORDS + k - 1];
            oi[k] = lds[v * OSCQ_GWORDS + MAXK + k - 1];
        }
        phase += lds[v * OSCQ_GWORDS + 2 * MAXK];
        cpmul<K>(Sr, Si, orr, oi);
        if (v < w) cpmul<K>(wpr, wpi, orr, oi);
        if (v > w) cpmul<K>(wsr, wsi, orr, oi);
    }
    cpmul<K>(pr, pi, wpr, wpi);
    cpmul<K>(sr, si, wsr, wsi);

    double s_re = 1.0, s_im = 0.0;
#pragma unroll
    for (int k = K; k >= 1; --k) { s_re += Sr[k]; s_im += Si[k]; }
    double sn, cs;
    sincos(phase, &sn, &cs);
    if (tid == 0) grad[q.param_offset] = g * (-2.0 * 3.141592653589793 * fma(sn, s_re, cs * s_im));

    // pass 2: per coordinate R_t, G_t, the derivative surpluses and the two
    // gradient entries
    for (int t = tid; t < d; t += 256) {
        double Rr[MAXK + 1], Ri[MAXK + 1];
#pragma unroll
        for (int k = 0; k <= MAXK; ++k) { Rr[k] = pr[k]; Ri[k] = pi[k]; }
        cpmul<K>(Rr, Ri, sr, si);
        if (!single) {
            for (int t2 = tid; t2 < d; t2 += 256) {
                if (t2 == t) continue;
                double orr[MAXK + 1], oi[MAXK + 1];
                orr[0] = 0.0;
                oi[0] = 0.0;
#pragma unroll
                for (int k = 1; k <= K; ++k) {
                    orr[k] = wsp[(size_t)t2 * 2 * K + 2 * (k - 1)];
                    oi[k] = wsp[(size_t)t2 * 2 * K + 2 * (k - 1) + 1];
                }
                cpmul<K>(Rr, Ri, orr, oi);
            }
        }
        // G[e] = sum_{j <= K-e} R[j], R[0] = 1
        double Gr[MAXK + 1], Gi[MAXK + 1];
        {
            double cr = 1.0, ci = 0.0;
            Gr[K] = 1.0;
            Gi[K] = 0.0;
#pragma unroll
            for (int e = K - 1; e >= 1; --e) {
                cr += Rr[K - e];
                ci += Ri[K - e];
                Gr[e] = cr;
                Gi[e] = ci;
            }
        }
        const double a = prm[1 + t], hv = 0.5 - prm[1 + d + t];
        double ar[MAXK + 1], ai[MAXK + 1], ur[MAXK + 1], ui[MAXK + 1];
        int opaque = 0;
        asm volatile("" : "+s"(opaque));
        dsurplus_oscq<K, RC>(r64 + opaque, a, 2.0 * hv, ar, ai, ur, ui);
        double da_r = 0.0, da_i = 0.0, du_r = 0.0, du_i = 0.0;
#pragma unroll
        for (int e = 1; e <= K; ++e) {
            da_r = fma(Gr[e], ar[e], fma(-Gi[e], ai[e], da_r));
            da_i = fma(Gr[e], ai[e], fma(Gi[e], ar[e], da_i));
            du_r = fma(Gr[e], ur[e], fma(-Gi[e], ui[e], du_r));
            du_i = fma(Gr[e], ui[e], fma(Gi[e], ur[e], du_i));
        }
        // Z = i dPhi S + dS; dQ = Re(E Z) = cos Phi Re Z - sin Phi Im Z
        const double pa = hv * hv, pu = -2.0 * a * hv;
        const double za_r = da_r - pa * s_im, za_i = da_i + pa * s_re;
        const double zu_r = du_r - pu * s_im, zu_i = du_i + pu * s_re;
        grad[q.param_offset + 1 + t] = g * fma(cs, za_r, -sn * za_i);
        grad[q.param_offset + 1 + d + t] = g * fma(cs, zu_r, -sn * zu_i);
    }
}

__global__ void __launch_bounds__(256)
k_oscq_grad(const OscqDesc* __restrict__ descs, const double* __restrict__ pool64,
            const double* __restrict__ params, const double* __restrict__ gout, double* __restrict__ grad,
            double* __restrict__ ws)
{
    __shared__ double lds[4 * OSCQ_GWORDS];
    const OscqDesc q = descs[blockIdx.x];
    const int K = __builtin_amdgcn_readfirstlane(q.K);
    const int rc = __builtin_amdgcn_readfirstlane(rule_class_of(q.rule));
    const double* r64 = pool64 + q.off64;
    const double* prm = params + q.param_offset;
    const double g = gout[q.out_index];
    switch_k<MAXK>(K, [&](auto kc) {
        constexpr int KK = decltype(kc)::value;
        if (rc == RC_NESTED) oscq_grad_body<KK, RC_NESTED>(q, r64, prm, g, grad, ws, lds);
        else if (rc == RC_GL2) oscq_grad_body<KK, RC_GL2>(q, r64, prm, g, grad, ws, lds);
        else if (rc == RC_GP) oscq_grad_body<KK, RC_GP>(q, r64, prm, g, grad, ws, lds);
        else oscq_grad_body<KK, RC_GLP>(q, r64, prm, g, grad, ws, lds);
    });
}

}  // namespace dev

int launch_oscq(int d, int K, int rule, int G, const double* pool64, const double* params, double* out,
                double* bound, double* scratch, void* stream)
{
    hipLaunchKernelGGL(dev::k_oscq, dim3((unsigned)G), dim3(256), 0, (hipStream_t)stream, d, K, rule, G, pool64,
                       params, out, bound, scratch);
    return (int)hipGetLastError();
}

int launch_oscq_batch(int n, const OscqDesc* descs, const double* pool64, const double* params, double* out,
                      double* bound, void* stream)
{
    if (n <= 0) return 0;
    hipLaunchKernelGGL(dev::k_oscq_batch, dim3((unsigned)n), dim3(256), 0, (hipStream_t)stream, descs, pool64,
                       params, out, bound);
    return (int)hipGetLastError();
}

}  // namespace sg

namespace sg {

int launch_oscq_grad(int n, const OscqDesc* descs, const double* pool64, const double* params, const double* gout,
                     double* grad, double* ws, void* stream)
{
    if (n <= 0) return 0;
    hipLaunchKernelGGL(dev::k_oscq_grad, dim3((unsigned)n), dim3(256), 0, (hipStream_t)stream, descs, pool64, params,
                       gout, grad, ws);
    return (int)hipGetLastError();
}

}  // namespace sg
