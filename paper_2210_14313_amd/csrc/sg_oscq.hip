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
// One workgroup of 256 threads per integrand (a plan launches one per
// oscillatory-quadratic integrand): each thread sweeps the
// coordinates t = tid, tid + 256, ..., a wave combines its lanes by an
// xor butterfly of complex truncated products, and the first thread joins
// the four waves in wave order and reads out the value and its bound.
#include "sg_device.hpp"
#include "sg_oscq.hpp"

namespace sg {
namespace dev {

constexpr int OSCQ_WORDS = 2 * MAXK + 4;   // doubles per wave in LDS

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

template <int K, int RC>
__device__ void oscq_body(int d, const double* __restrict__ r64, const double* __restrict__ prm,
                          double* __restrict__ out, double* __restrict__ bound, double* lds)
{
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    double ar[MAXK + 1], ai[MAXK + 1];
#pragma unroll
    for (int k = 0; k <= MAXK; ++k) { ar[k] = 0.0; ai[k] = 0.0; }
    double m = 0.0, eps = 0.0, ph = 0.0, phabs = 0.0;
    for (int t = tid; t < d; t += 256) {
        const double a = prm[1 + t], hv = 0.5 - prm[1 + d + t];
        double dr[MAXK + 1], di[MAXK + 1], e_t = 0.0;
        int opaque = 0;
        asm volatile("" : "+s"(opaque));
        surplus_oscq<K, RC>(r64 + opaque, a, 2.0 * hv, dr, di, e_t);
        cpmul<K>(ar, ai, dr, di);
        double mt = 0.0;
#pragma unroll
        for (int k = 1; k <= K; ++k) mt += fabs(dr[k]) + fabs(di[k]);
        m += mt;
        eps += e_t;
        const double term = a * (hv * hv);          // phase of g_t(1/2)
        ph += term;
        phabs += fabs(term);
    }
    for (int off = 32; off >= 1; off >>= 1) {
        double br[MAXK + 1], bi[MAXK + 1];
#pragma unroll
        for (int k = 1; k <= K; ++k) {
            br[k] = __shfl_xor(ar[k], off);
            bi[k] = __shfl_xor(ai[k], off);
        }
        cpmul<K>(ar, ai, br, bi);
        m += __shfl_xor(m, off);
        eps += __shfl_xor(eps, off);
        ph += __shfl_xor(ph, off);
        phabs += __shfl_xor(phabs, off);
    }
    if (lane == 0) {
        double* s = lds + w * OSCQ_WORDS;
#pragma unroll
        for (int k = 1; k <= K; ++k) {
            s[k - 1] = ar[k];
            s[MAXK + k - 1] = ai[k];
        }
        s[2 * MAXK] = m;
        s[2 * MAXK + 1] = eps;
        s[2 * MAXK + 2] = ph;
        s[2 * MAXK + 3] = phabs;
    }
    __syncthreads();
    if (tid != 0) return;
    for (int v = 1; v < 4; ++v) {
        const double* s = lds + v * OSCQ_WORDS;
        double br[MAXK + 1], bi[MAXK + 1];
#pragma unroll
        for (int k = 1; k <= K; ++k) {
            br[k] = s[k - 1];
            bi[k] = s[MAXK + k - 1];
        }
        cpmul<K>(ar, ai, br, bi);
        m += s[2 * MAXK];
        eps += s[2 * MAXK + 1];
        ph += s[2 * MAXK + 2];
        phabs += s[2 * MAXK + 3];
    }
    double sr = 0.0, si = 0.0;
#pragma unroll
    for (int k = K; k >= 1; --k) {
        sr += ar[k];
        si += ai[k];
    }
    sr += 1.0;
    const double wp = 2.0 * 3.141592653589793 * prm[0];
    const double phase = wp + ph;
    double sn, cs;
    sincos(phase, &sn, &cs);
    const double Q = fma(cs, sr, -sn * si);
    out[0] = Q;
    if (bound) {
        const double u64 = 1.1102230246251565e-16;
        // coefficients of every partial product are bounded in sum by
        // exp(sum_t sum_e |delta_t[e]|) (as for the real sweep)
        const double sabs = exp(m) * (1.0 + 1e-13);
        // pair values: 8 roundings relative to mag; within-rule sums: one
        // FMA chain over the table's pairs
        const double rel = u64 * (8.0 + (double)total_pairs<RC, K>());
        // product tree: a thread's ceil(d/256) coordinates, 6 butterfly
        // levels, 3 wave joins; a complex truncated product rounds each
        // component at most 2K + 2 times
        const double levels = (double)((d + 255) / 256 + 9);
        const double dsum = sabs * (rel * eps + (2.0 * K + 4.0) * levels * u64);
        // phase: d - 1 additions of terms rounded twice each, and 2 pi w
        const double ph_err = u64 * (double)(d + 3) * phabs + 2.0 * u64 * fabs(wp);
        const double smag = sqrt(fma(sr, sr, si * si)) + dsum;
        bound[0] = dsum + smag * (ph_err + u64 * (fabs(phase) + 8.0));
    }
}

__device__ __forceinline__ void oscq_dispatch(int d, int K, int rule, const double* r64, const double* prm,
                                              double* out, double* bound, double* lds)
{
    const int rc = rule_class_of(rule);
    switch_k<MAXK>(K, [&](auto kc) {
        constexpr int KK = decltype(kc)::value;
        if (rc == RC_NESTED) oscq_body<KK, RC_NESTED>(d, r64, prm, out, bound, lds);
        else if (rc == RC_GL2) oscq_body<KK, RC_GL2>(d, r64, prm, out, bound, lds);
        else if (rc == RC_GP) oscq_body<KK, RC_GP>(d, r64, prm, out, bound, lds);
        else oscq_body<KK, RC_GLP>(d, r64, prm, out, bound, lds);
    });
}

__global__ void __launch_bounds__(256)
k_oscq(int d, int K, int rule, const double* __restrict__ pool64, const double* __restrict__ params,
       double* __restrict__ out, double* __restrict__ bound)
{
    __shared__ double lds[4 * OSCQ_WORDS];
    oscq_dispatch(d, K, rule, pool64, params, out, bound, lds);
}

// Workgroup b runs descriptor b.
__global__ void __launch_bounds__(256)
k_oscq_batch(const OscqDesc* __restrict__ descs, const double* __restrict__ pool64,
             const double* __restrict__ params, double* __restrict__ out, double* __restrict__ bound)
{
    __shared__ double lds[4 * OSCQ_WORDS];
    const OscqDesc q = descs[blockIdx.x];
    oscq_dispatch(q.d, q.K, q.rule, pool64 + q.off64, params + q.param_offset, out + q.out_index,
                  bound ? bound + q.out_index : nullptr, lds);
}

}  // namespace dev

int launch_oscq(int d, int K, int rule, const double* pool64, const double* params, double* out, double* bound,
                void* stream)
{
    hipLaunchKernelGGL(dev::k_oscq, dim3(1), dim3(256), 0, (hipStream_t)stream, d, K, rule, pool64, params, out,
                       bound);
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
