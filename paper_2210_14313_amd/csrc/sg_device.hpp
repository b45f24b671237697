#pragma once
// Device code (gfx950) of the Smolyak dimension sweep, included by the
// per-precision kernel units sg_fwd*.hip / sg_adj*.hip / sg_unrank.hip.
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

#include <type_traits>

#include "sg_internal.hpp"
#include "sg_math.hpp"
#include "sg_tables.inc"

namespace sg {
namespace dev {

constexpr int MAXK = kMaxK;
constexpr int FAM_EXP = SG_FAMILY_EXP_SUM;
constexpr int FAM_OSC = SG_FAMILY_OSCILLATORY;
constexpr int FAM_PEAK = SG_FAMILY_PRODUCT_PEAK;
constexpr int FAM_GAUSS = SG_FAMILY_GAUSSIAN;

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

// The same series on |v| <= 1 (z <= 1), used by the compiled-table path
// whenever |parameter| <= 2 (every node has y <= 1/2).  First dropped term
// relative to 1: 2/20! < 1e-18 (FP64, 9 terms) and 2/12! < 5e-9 (FP32, 5 terms).
__device__ __forceinline__ double series64w(double z)
{
    double p = 1.0 / 3201186852864000.0;              // 2/18!
    p = fma(p, z, 1.0 / 10461394944000.0);             // 2/16!
    p = fma(p, z, 1.0 / 43589145600.0);                // 2/14!
    p = fma(p, z, 1.0 / 239500800.0);                  // 2/12!
    p = fma(p, z, 1.0 / 1814400.0);                    // 2/10!
    p = fma(p, z, 1.0 / 20160.0);                      // 2/8!
    p = fma(p, z, 1.0 / 360.0);                        // 2/6!
    p = fma(p, z, 1.0 / 12.0);                         // 2/4!
    p = fma(p, z, 1.0);                                // 2/2!
    return p;
}

__device__ __forceinline__ float series32w(float z)
{
    float p = 1.0f / 1814400.0f;
    p = fmaf(p, z, 1.0f / 20160.0f);
    p = fmaf(p, z, 1.0f / 360.0f);
    p = fmaf(p, z, 1.0f / 12.0f);
    p = fmaf(p, z, 1.0f);
    return p;
}

// sinh(v)/v = sum z^k/(2k+1)! (z = v^2; sin(v)/v with z = -v^2) on |v| <= 1,
// for the compiled-table reverse sweep: first dropped term relative to 1: 1/21! < 2e-20 (FP64, 10 terms),
// 1/13! < 2e-10 (FP32, 6 terms).
__device__ __forceinline__ double series_s64w(double z)
{
    double p = 1.0 / 121645100408832000.0;             // 1/19!
    p = fma(p, z, 1.0 / 355687428096000.0);            // 1/17!
    p = fma(p, z, 1.0 / 1307674368000.0);              // 1/15!
    p = fma(p, z, 1.0 / 6227020800.0);                 // 1/13!
    p = fma(p, z, 1.0 / 39916800.0);                   // 1/11!
    p = fma(p, z, 1.0 / 362880.0);                     // 1/9!
    p = fma(p, z, 1.0 / 5040.0);                       // 1/7!
    p = fma(p, z, 1.0 / 120.0);                        // 1/5!
    p = fma(p, z, 1.0 / 6.0);                          // 1/3!
    p = fma(p, z, 1.0);
    return p;
}

__device__ __forceinline__ float series_s32w(float z)
{
    float p = 1.0f / 39916800.0f;                      // 1/11!
    p = fmaf(p, z, 1.0f / 362880.0f);
    p = fmaf(p, z, 1.0f / 5040.0f);
    p = fmaf(p, z, 1.0f / 120.0f);
    p = fmaf(p, z, 1.0f / 6.0f);
    p = fmaf(p, z, 1.0f);
    return p;
}

// Per-coordinate family parameters, read once per coordinate.
struct CoordParam {
    double p0;    // exp: c; osc: a; peak: beta = b^-2; gaussian: c
    double p1;    // peak: (1 - 2u)/2; gaussian: c (1 - 2u)
};

// Gaussian exp(c (x - u)^2): with b = 1 - 2u, h(y) = g(1/2 + y)/g(1/2) - 1 =
// e^{c y (y + b)} - 1 and h(y) + h(-y) = 2 (e^{c y^2} cosh(c b y) - 1) =
// 2 (E (1 + C) + C), E = expm1(c y^2), C = cosh(c b y) - 1 = F^2 / (2 (1 + F))
// with F = expm1(|c b y|) (no cancellation).  For c < 0 the two terms have
// opposite signs and may cancel, so the value's rounding is charged against
// the magnitude 2 (|E| (1 + C) + C), returned in `mag` (E and F carry at most
// 5 roundings each, C three more, the combination two more).  Branch-free
// expm1 keeps the code small: this family takes the table-driven path only.
__device__ __forceinline__ double pair_gauss64(const CoordParam& cp, double y, double& mag)
{
    const double E = expm1_any(cp.p0 * (y * y));
    const double F = expm1_any(fabs(cp.p1 * y));
    const double C = 0.5 * (F * (F / (1.0 + F)));
    mag = 2.0 * fma(fabs(E), 1.0 + C, C);
    return 2.0 * fma(E, 1.0 + C, C);
}

// A pair value with the magnitude its rounding is charged against (the
// Gaussian's); plain values are their own magnitude.
struct PairVM {
    double v, m;
};
struct PairVMf {
    float v, m;
};
__device__ __forceinline__ double pv_val(double s) { return s; }
__device__ __forceinline__ double pv_mag(double s) { return fabs(s); }
__device__ __forceinline__ double pv_val(const PairVM& s) { return s.v; }
__device__ __forceinline__ double pv_mag(const PairVM& s) { return s.m; }
__device__ __forceinline__ float pv_val(float s) { return s; }
__device__ __forceinline__ float pv_mag(float s) { return fabsf(s); }
__device__ __forceinline__ float pv_val(const PairVMf& s) { return s.v; }
__device__ __forceinline__ float pv_mag(const PairVMf& s) { return s.m; }

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
    } else if constexpr (FAM == FAM_GAUSS) {
        double mag;
        return pair_gauss64(cp, y, mag);
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
        if (fabsf(v) <= 1.0f) {
            const float z = FAM == FAM_EXP ? v * v : -(v * v);
            return z * series32w(z);
        }
    }
    // Outside the series range (and for the product-peak family, a rational
    // function whose cancellation-prone parts need the wider format) the
    // value is formed in FP64 and rounded once, so every pair value carries
    // at most the series path's relative error whatever the parameter.
    return (float)pair64<FAM>(cp, y);
}

// Pair values on the compiled-table path, |c| <= 2 so |v| <= 1.  The series
// only needs z = +-(c y)^2, formed as (+-c^2) * y^2 with the per-coordinate
// factor c2s = +-c^2 rounded once and y^2 a per-pair constant (split into two
// FP32 constants in FP32, so no systematic per-node rounding enters).
template <int FAM, bool SPLIT>
__device__ __forceinline__ float pair32_z(float c2s, float y2h, float y2l)
{
    const float z = SPLIT ? fmaf(c2s, y2h, c2s * y2l) : c2s * y2h;
    return z * series32w(z);
}

__device__ __forceinline__ double pair64_z(double c2s, double y2)
{
    const double z = c2s * y2;
    return z * series64w(z);
}

// +-c^2 for the series argument z (exp-sum: +, oscillatory: -).
template <int FAM>
__device__ __forceinline__ double signed_c2(double c)
{
    return FAM == FAM_EXP ? c * c : -(c * c);
}

// The FP32 series of a coordinate use z = c2s y^2 with c2s the per-coordinate
// factor +-c^2 rounded once to FP32, i.e. every pair value of the coordinate
// has its argument off by the same relative amount r = (c2 - c2s) / c2s.
// With s(z) = z P(z), s(z (1 + r)) = s(z) (1 + r + r z P'(z)/P(z) + O(r^2)),
// so scaling the coordinate's surpluses by 1 + r removes that error up to a
// remainder of relative size |r| z / 12 <= 2^-24 / 12 (z <= 1 on this path).
template <int FAM, int K>
__device__ __forceinline__ void argument_correction(double c, float c2s, double (&del)[MAXK + 1])
{
    // |r| <= 2^-24, so a reciprocal good to a few FP32 units leaves r
    // accurate far below the FP64 rounding of the surpluses
    const double c2 = signed_c2<FAM>(c);
    const double r = c2s != 0.0f ? (c2 - (double)c2s) * (double)__builtin_amdgcn_rcpf(c2s) : 0.0;
#pragma unroll
    for (int e = 1; e <= K; ++e) del[e] = fma(del[e], r, del[e]);
}

// Compensated FP32 accumulation of w*s with w = wh + wl: two-sum of the
// rounded product into the running sum (its error goes to lo, exactly), and
// the low weight part w_l*s added to lo.  Each product keeps its own
// rounding (half an ulp, independent between terms, the size of the pair
// value's own rounding); the bound accounts for it.
__device__ __forceinline__ void acc2(float& hi, float& lo, float wh, float wl, float s)
{
    const float p = wh * s;
    const float t = hi + p;
    const float bp = t - hi;
    const float err = (hi - (t - bp)) + (p - bp);
    hi = t;
    lo = fmaf(wl, s, lo + err);
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
// Compile-time loop over the levels L = B .. E-1.
template <int B, int E, class F>
__device__ __forceinline__ void static_for(F&& f)
{
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        static_for<B + 1, E>(f);
    }
}

// delta_t[e] for one coordinate, FP64.  The table is a sequence of per-pair
// records (y, dW[elo..ehi], sum|dW|) whose layout is fixed by (RC, K), so
// every load has a compile-time offset from the table base.  `pf` maps the
// pair's y to its (even-part) value.
template <int K, int RC, class PF>
__device__ __forceinline__ void surplus64g(const double* __restrict__ r64, PF&& pf, bool want_bound,
                                           double (&del)[MAXK + 1], double& eps)
{
#pragma unroll
    for (int e = 0; e <= MAXK; ++e) del[e] = 0.0;
    static_for<2, K + 2>([&](auto Lc) {
        constexpr int L = decltype(Lc)::value;
        constexpr int np = rc_pairs(RC, L), lo = rc_elo(L), hi = rc_ehi(RC, K, L);
        constexpr int rl = rc_rec64(RC, K, L), off = rc_off64(RC, K, L);
#pragma unroll 2
        for (int j = 0; j < np; ++j) {
            const double* r = r64 + off + j * rl;
            const auto sr = pf(r[0]);
            const double s = pv_val(sr);
#pragma unroll
            for (int e = lo; e <= hi; ++e) del[e] = fma(r[1 + e - lo], s, del[e]);
            if (want_bound) eps = fma(r[rl - 1], pv_mag(sr), eps);
        }
    });
}

// Same with FP32 pair values and two-sum compensated FP32 accumulation
// against hi+lo weights; emitted as FP64 hi + lo.
template <int K, int RC, class PF>
__device__ __forceinline__ void surplus32g(const double* __restrict__ r64, const float* __restrict__ r32,
                                           PF&& pf, bool want_bound, double (&del)[MAXK + 1], double& eps)
{
    float hi[MAXK + 1], lo[MAXK + 1];
#pragma unroll
    for (int e = 0; e <= MAXK; ++e) { hi[e] = 0.0f; lo[e] = 0.0f; }
    float epsf = 0.0f;
    static_for<2, K + 2>([&](auto Lc) {
        constexpr int L = decltype(Lc)::value;
        constexpr int np = rc_pairs(RC, L), elo = rc_elo(L), ehi = rc_ehi(RC, K, L);
        constexpr int rl = rc_rec64(RC, K, L), off = rc_off64(RC, K, L);
        constexpr int rl32 = rc_rec32(RC, K, L), off32 = rc_off32(RC, K, L);
#pragma unroll 2
        for (int j = 0; j < np; ++j) {
            const double* r = r64 + off + j * rl;
            const float* w = r32 + off32 + j * rl32;
            const auto sr = pf(r[0]);
            const float s = pv_val(sr);
#pragma unroll
            for (int e = elo; e <= ehi; ++e)
                acc2(hi[e], lo[e], w[2 * (e - elo)], w[2 * (e - elo) + 1], s);
            if (want_bound) epsf = fmaf((float)r[rl - 1], pv_mag(sr), epsf);
        }
    });
#pragma unroll
    for (int e = 0; e <= MAXK; ++e) del[e] = (double)hi[e] + (double)lo[e];
    eps += (double)epsf;
}

template <int K, int RC, int FAM>
__device__ __forceinline__ void surplus64(const double* __restrict__ r64, const CoordParam& cp, bool want_bound,
                                          double (&del)[MAXK + 1], double& eps)
{
    if constexpr (FAM == FAM_GAUSS)
        surplus64g<K, RC>(r64, [&](double y) { PairVM p; p.v = pair_gauss64(cp, y, p.m); return p; }, want_bound,
                          del, eps);
    else
        surplus64g<K, RC>(r64, [&](double y) { return pair64<FAM>(cp, y); }, want_bound, del, eps);
}

template <int K, int RC, int FAM>
__device__ __forceinline__ void surplus32(const double* __restrict__ r64, const float* __restrict__ r32,
                                          const CoordParam& cp, bool want_bound, double (&del)[MAXK + 1],
                                          double& eps)
{
    if constexpr (FAM == FAM_GAUSS)
        surplus32g<K, RC>(r64, r32, [&](double y) {
            double m;
            const double v = pair_gauss64(cp, y, m);
            PairVMf p;
            p.v = (float)v;
            p.m = (float)m;
            return p;
        }, want_bound, del, eps);
    else
        surplus32g<K, RC>(r64, r32, [&](double y) { return pair32<FAM>(cp, y); }, want_bound, del, eps);
}

// ------------------------------------------- compiled-table surpluses
// For K <= KCONST the record tables of every rule are compiled into the
// kernels (sg_tables.inc, written at build time by the same host code that
// builds the run-time tables), so each node and weight is an instruction
// constant: no table loads and no waits on them in the coordinate loop.
constexpr int KCONST = 6;

// First pair index of level L in the pair order.
template <int RC>
constexpr int pair_base(int L)
{
    int n = 0;
    for (int l = 2; l < L; ++l) n += rc_pairs(RC, l);
    return n;
}

// Lowest level whose pairs carry weight in row e (rows are filled first by
// that level's first pair).
template <int RC, int K>
constexpr int first_level(int e)
{
    for (int L = 2; L <= K + 1; ++L)
        if (rc_pairs(RC, L) > 0 && rc_elo(L) <= e && e <= rc_ehi(RC, K, L)) return L;
    return -1;
}

// The pair with the largest y (level, index) and the sum of |dW| over all
// pairs and rows of a (rule, K) table.  For the exp-sum and oscillatory
// families |s(y)| grows with y on the series range, so
// sum_p (sum_e |dW[e][p]|) |s_p| <= total_wabs * |s(y_max)|: the bound's
// per-coordinate term costs one multiply instead of one per pair.
template <int RULE, int K>
struct TableFacts {
    static constexpr int RC = rule_class_of(RULE);
    using R = tab::Rec<RULE, K>;
    static constexpr int max_pair()
    {
        int best = -1;
        double by = -1.0;
        int p = 0;
        for (int L = 2; L <= K + 1; ++L)
            for (int J = 0; J < rc_pairs(RC, L); ++J, ++p) {
                const double y = R::r64[rc_off64(RC, K, L) + J * rc_rec64(RC, K, L)];
                if (y > by) { by = y; best = p; }
            }
        return best;
    }
    static constexpr double total_wabs()
    {
        double w = 0.0;
        for (int L = 2; L <= K + 1; ++L)
            for (int J = 0; J < rc_pairs(RC, L); ++J)
                w += R::r64[rc_off64(RC, K, L) + J * rc_rec64(RC, K, L) + rc_rec64(RC, K, L) - 1];
        return w * (1.0 + 1.0 / 1048576.0);   // margin for the rounding of the sum and of s(y_max)
    }
};

// FP64: delta_t[e] = sum_p dW[e][p] s_p with every (y, dW, sum|dW|) a
// compile-time constant.  `fast` lanes (|c| <= 2, and every product-peak
// lane) use the series / rational forms; the caller sends other lanes to
// the table-driven path.
template <int RULE, int K, int FAM>
__device__ __forceinline__ void surplus64_const(const CoordParam& cp, double (&del)[MAXK + 1], double& eps)
{
    constexpr int RC = rule_class_of(RULE);
    using R = tab::Rec<RULE, K>;
#pragma unroll
    for (int e = 0; e <= MAXK; ++e) del[e] = 0.0;
    double et = 0.0;
    const double c2s = signed_c2<FAM>(cp.p0);
    static_for<2, K + 2>([&](auto Lc) {
        constexpr int L = decltype(Lc)::value;
        constexpr int off = rc_off64(RC, K, L), rl = rc_rec64(RC, K, L);
        constexpr int lo = rc_elo(L), hi = rc_ehi(RC, K, L);
        static_for<0, rc_pairs(RC, L)>([&](auto Jc) {
            constexpr int J = decltype(Jc)::value;
            constexpr double y = R::r64[off + J * rl];
            double sv;
            if constexpr (FAM == FAM_PEAK) sv = pair64<FAM_PEAK>(cp, y);
            else sv = pair64_z(c2s, y * y);
            static_for<lo, hi + 1>([&](auto Ec) {
                constexpr int E = decltype(Ec)::value;
                constexpr double w = R::r64[off + J * rl + 1 + E - lo];
                if constexpr (first_level<RC, K>(E) == L && J == 0) del[E] = w * sv;
                else del[E] = fma(w, sv, del[E]);
            });
            if constexpr (FAM == FAM_PEAK) {
                constexpr double wa = R::r64[off + J * rl + rl - 1];
                et = fma(wa, fabs(sv), et);
            } else if constexpr (pair_base<RC>(L) + J == TableFacts<RULE, K>::max_pair()) {
                // (a constexpr variable: the table walk must not run per coordinate)
                constexpr double wt = TableFacts<RULE, K>::total_wabs();
                et = wt * fabs(sv);
            }
        });
    });
    eps += et;
}

// Position of the pair (L, J) among the terms of row e (pairs in level
// order) and the length of row e.
template <int RC, int K>
constexpr int row_index(int e, int L, int J)
{
    int n = 0;
    for (int l = 2; l < L; ++l)
        if (rc_elo(l) <= e && e <= rc_ehi(RC, K, l)) n += rc_pairs(RC, l);
    return n + J;
}
template <int RC, int K>
constexpr int row_length(int e)
{
    int n = 0;
    for (int l = 2; l <= K + 1; ++l)
        if (rc_elo(l) <= e && e <= rc_ehi(RC, K, l)) n += rc_pairs(RC, l);
    return n;
}

// Terms per block of the blocked two-sum below.
constexpr int kSumBlock = 8;

// hi + lo += b with the rounding error of the addition kept exactly (two-sum).
__device__ __forceinline__ void two_sum_into(float& hi, float& lo, float b)
{
    const float t = hi + b;
    const float bp = t - hi;
    const float err = (hi - (t - bp)) + (b - bp);
    hi = t;
    lo += err;
}

// FP32 pair values, compensated FP32 sums against hi+lo weights: the high
// weight parts are summed by an FMA chain over blocks of kSumBlock
// consecutive terms of a row, the block sums enter the row's (hi, lo) pair by
// two-sum, and the low weight parts go to lo by FMA.  Per term 2 + 6/kSumBlock
// instructions; the rounding of a block's chain (at most kSumBlock roundings
// of partial sums of its terms) is what the error bound charges per term.
template <int RULE, int K, int FAM>
__device__ __forceinline__ void surplus32_const(const CoordParam& cp, double (&del)[MAXK + 1], double& eps)
{
    constexpr int RC = rule_class_of(RULE);
    using R = tab::Rec<RULE, K>;
    float hi[MAXK + 1], lo[MAXK + 1], part[MAXK + 1];
#pragma unroll
    for (int e = 0; e <= MAXK; ++e) { hi[e] = 0.0f; lo[e] = 0.0f; part[e] = 0.0f; }
    float epsf = 0.0f;
    const float c2s = (float)signed_c2<FAM>(cp.p0);
    static_for<2, K + 2>([&](auto Lc) {
        constexpr int L = decltype(Lc)::value;
        constexpr int off = rc_off64(RC, K, L), rl = rc_rec64(RC, K, L);
        constexpr int off32 = rc_off32(RC, K, L), rl32 = rc_rec32(RC, K, L);
        constexpr int elo = rc_elo(L), ehi = rc_ehi(RC, K, L);
        static_for<0, rc_pairs(RC, L)>([&](auto Jc) {
            constexpr int J = decltype(Jc)::value;
            constexpr double y = R::r64[off + J * rl];
            float sv;
            if constexpr (FAM == FAM_PEAK) {
                sv = (float)pair64<FAM_PEAK>(cp, y);
            } else {
                constexpr double y2 = y * y;
                constexpr float y2h = (float)y2;
                constexpr float y2l = (float)(y2 - (double)y2h);
                sv = pair32_z<FAM, y2l != 0.0f>(c2s, y2h, y2l);
            }
            static_for<elo, ehi + 1>([&](auto Ec) {
                constexpr int E = decltype(Ec)::value;
                constexpr float wh = R::r32[off32 + J * rl32 + 2 * (E - elo)];
                constexpr float wl = R::r32[off32 + J * rl32 + 2 * (E - elo) + 1];
                constexpr int k = row_index<RC, K>(E, L, J), n = row_length<RC, K>(E);
                constexpr bool block_end = (k % kSumBlock == kSumBlock - 1) || (k == n - 1);
                if constexpr (k % kSumBlock == 0) part[E] = wh * sv;
                else part[E] = fmaf(wh, sv, part[E]);
                if constexpr (k == 0) lo[E] = wl * sv;
                else lo[E] = fmaf(wl, sv, lo[E]);
                if constexpr (block_end) {
                    if constexpr (k < kSumBlock) hi[E] = part[E];
                    else two_sum_into(hi[E], lo[E], part[E]);
                }
            });
            if constexpr (FAM == FAM_PEAK) {
                constexpr float wa = (float)R::r64[off + J * rl + rl - 1];
                epsf = fmaf(wa, fabsf(sv), epsf);
            } else if constexpr (pair_base<RC>(L) + J == TableFacts<RULE, K>::max_pair()) {
                constexpr float wt = (float)TableFacts<RULE, K>::total_wabs();
                epsf = wt * fabsf(sv);
            }
        });
    });
#pragma unroll
    for (int e = 0; e <= MAXK; ++e) del[e] = (double)hi[e] + (double)lo[e];
    if constexpr (FAM != FAM_PEAK) argument_correction<FAM, K>(cp.p0, c2s, del);
    eps += (double)epsf;
}

// FP32 pair values accumulated against FP64 weights in FP64 (on CDNA4 an
// FP64 FMA issues at the FP32 rate, so the wider accumulator costs one
// instruction per term where the two-sum costs eight).
template <int RULE, int K, int FAM>
__device__ __forceinline__ void surplus32e_const(const CoordParam& cp, double (&del)[MAXK + 1], double& eps)
{
    constexpr int RC = rule_class_of(RULE);
    using R = tab::Rec<RULE, K>;
#pragma unroll
    for (int e = 0; e <= MAXK; ++e) del[e] = 0.0;
    float epsf = 0.0f;
    const float c2s = (float)signed_c2<FAM>(cp.p0);
    static_for<2, K + 2>([&](auto Lc) {
        constexpr int L = decltype(Lc)::value;
        constexpr int off = rc_off64(RC, K, L), rl = rc_rec64(RC, K, L);
        constexpr int lo = rc_elo(L), hi = rc_ehi(RC, K, L);
        static_for<0, rc_pairs(RC, L)>([&](auto Jc) {
            constexpr int J = decltype(Jc)::value;
            constexpr double y = R::r64[off + J * rl];
            float sv;
            if constexpr (FAM == FAM_PEAK) {
                sv = (float)pair64<FAM_PEAK>(cp, y);
            } else {
                constexpr double y2 = y * y;
                constexpr float y2h = (float)y2;
                constexpr float y2l = (float)(y2 - (double)y2h);
                sv = pair32_z<FAM, y2l != 0.0f>(c2s, y2h, y2l);
            }
            const double sd = (double)sv;
            static_for<lo, hi + 1>([&](auto Ec) {
                constexpr int E = decltype(Ec)::value;
                constexpr double w = R::r64[off + J * rl + 1 + E - lo];
                if constexpr (first_level<RC, K>(E) == L && J == 0) del[E] = w * sd;
                else del[E] = fma(w, sd, del[E]);
            });
            if constexpr (FAM == FAM_PEAK) {
                constexpr float wa = (float)R::r64[off + J * rl + rl - 1];
                epsf = fmaf(wa, fabsf(sv), epsf);
            } else if constexpr (pair_base<RC>(L) + J == TableFacts<RULE, K>::max_pair()) {
                constexpr float wt = (float)TableFacts<RULE, K>::total_wabs();
                epsf = wt * fabsf(sv);
            }
        });
    });
    if constexpr (FAM != FAM_PEAK) argument_correction<FAM, K>(cp.p0, c2s, del);
    eps += (double)epsf;
}

// Derivative surpluses d delta_t[e] / d c_t of the exp-sum (c) and
// oscillatory (a) families on the compiled-table path (|c| <= 2): per pair
// ds/dc = +-2 c y^2 S(+-c^2 y^2), S(z) = sinh(v)/v or sin(v)/v, against the
// compile-time difference weights.  FP64: an FMA chain per row; FP32: the
// blocked two-sum of the forward sweep against hi+lo weights.
template <int RULE, int K, int FAM>
__device__ __forceinline__ void dsurplus64_const(const CoordParam& cp, double (&dd)[MAXK + 1])
{
    constexpr int RC = rule_class_of(RULE);
    using R = tab::Rec<RULE, K>;
#pragma unroll
    for (int e = 0; e <= MAXK; ++e) dd[e] = 0.0;
    const double c2s = signed_c2<FAM>(cp.p0);
    const double f = (FAM == FAM_EXP ? 2.0 : -2.0) * cp.p0;
    static_for<2, K + 2>([&](auto Lc) {
        constexpr int L = decltype(Lc)::value;
        constexpr int off = rc_off64(RC, K, L), rl = rc_rec64(RC, K, L);
        constexpr int lo = rc_elo(L), hi = rc_ehi(RC, K, L);
        static_for<0, rc_pairs(RC, L)>([&](auto Jc) {
            constexpr int J = decltype(Jc)::value;
            constexpr double y = R::r64[off + J * rl];
            constexpr double y2 = y * y;
            const double dv = (f * y2) * series_s64w(c2s * y2);
            static_for<lo, hi + 1>([&](auto Ec) {
                constexpr int E = decltype(Ec)::value;
                constexpr double w = R::r64[off + J * rl + 1 + E - lo];
                if constexpr (first_level<RC, K>(E) == L && J == 0) dd[E] = w * dv;
                else dd[E] = fma(w, dv, dd[E]);
            });
        });
    });
}

template <int RULE, int K, int FAM>
__device__ __forceinline__ void dsurplus32_const(const CoordParam& cp, double (&dd)[MAXK + 1])
{
    constexpr int RC = rule_class_of(RULE);
    using R = tab::Rec<RULE, K>;
    float hi[MAXK + 1], lo[MAXK + 1], part[MAXK + 1];
#pragma unroll
    for (int e = 0; e <= MAXK; ++e) { hi[e] = 0.0f; lo[e] = 0.0f; part[e] = 0.0f; }
    const float c2s = (float)signed_c2<FAM>(cp.p0);
    const float f = (float)((FAM == FAM_EXP ? 2.0 : -2.0) * cp.p0);
    static_for<2, K + 2>([&](auto Lc) {
        constexpr int L = decltype(Lc)::value;
        constexpr int off = rc_off64(RC, K, L), rl = rc_rec64(RC, K, L);
        constexpr int off32 = rc_off32(RC, K, L), rl32 = rc_rec32(RC, K, L);
        constexpr int elo = rc_elo(L), ehi = rc_ehi(RC, K, L);
        static_for<0, rc_pairs(RC, L)>([&](auto Jc) {
            constexpr int J = decltype(Jc)::value;
            constexpr double y = R::r64[off + J * rl];
            constexpr double y2 = y * y;
            constexpr float y2h = (float)y2;
            constexpr float y2l = (float)(y2 - (double)y2h);
            const float z = y2l != 0.0f ? fmaf(c2s, y2h, c2s * y2l) : c2s * y2h;
            const float sv = (f * y2h) * series_s32w(z);
            static_for<elo, ehi + 1>([&](auto Ec) {
                constexpr int E = decltype(Ec)::value;
                constexpr float wh = R::r32[off32 + J * rl32 + 2 * (E - elo)];
                constexpr float wl = R::r32[off32 + J * rl32 + 2 * (E - elo) + 1];
                constexpr int k = row_index<RC, K>(E, L, J), n = row_length<RC, K>(E);
                constexpr bool block_end = (k % kSumBlock == kSumBlock - 1) || (k == n - 1);
                if constexpr (k % kSumBlock == 0) part[E] = wh * sv;
                else part[E] = fmaf(wh, sv, part[E]);
                if constexpr (k == 0) lo[E] = wl * sv;
                else lo[E] = fmaf(wl, sv, lo[E]);
                if constexpr (block_end) {
                    if constexpr (k < kSumBlock) hi[E] = part[E];
                    else two_sum_into(hi[E], lo[E], part[E]);
                }
            });
        });
    });
#pragma unroll
    for (int e = 0; e <= MAXK; ++e) dd[e] = (double)hi[e] + (double)lo[e];
}

// ----------------------------------------------------------- merge state
// Running polynomial a and the affine partial sum ls (FP64); for the error
// bound, m = sum_t sum_e |delta_t[e]|, eps = sum_t sum_p sum_e |dW[e][p]| |s_p|
// and lsabs = sum |terms of ls|.  The bound's sums have non-negative terms
// and are kept in FP32: a sum of n such terms rounded to nearest is at least
// (1 - n 2^-24) times the exact sum, which the read-out compensates
// (bound_sum_margin).
struct Acc {
    double a[MAXK + 1];
    double ls;
    float m, eps, lsabs;
};

template <int K>
__device__ __forceinline__ void acc_identity(Acc& x)
{
#pragma unroll
    for (int k = 0; k <= MAXK; ++k) x.a[k] = 0.0;
    x.ls = 0.0;
    x.m = x.eps = x.lsabs = 0.0f;
}

template <int K>
__device__ __forceinline__ void merge(Acc& x, const Acc& y, bool want_bound)
{
    pmul<K>(x.a, y.a);
    if (want_bound) {
        x.m += y.m;
        x.eps += y.eps;
        x.lsabs += y.lsabs;
    }
    x.ls += y.ls;
}

// Factor that makes an FP32 sum of at most n non-negative terms an upper
// bound of the exact sum: 1 / (1 - n 2^-24) <= 1 + 2 n 2^-24 for n < 2^22.
__device__ __forceinline__ double bound_sum_margin(int n)
{
    return 1.0 + (double)(2 * n + 2) * 5.9604644775390625e-08;
}

// DPP moves of a double (two 32-bit halves).  Lanes whose source is outside
// the pattern, or whose row is masked off, receive `fill`; with every row
// enabled (ROW_MASK 0xF) `fill` must be 0.0, which bound_ctrl supplies.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_f64(double v, double fill)
{
    const long long bv = __double_as_longlong(v), bf = __double_as_longlong(fill);
    int lo, hi;
    if constexpr (ROW_MASK == 0xF) {
        // every row enabled: with bound_ctrl set, a lane whose source lies
        // outside its row reads 0 (the identity's bits), no fill copy needed
        lo = __builtin_amdgcn_mov_dpp((int)bv, CTRL, 0xF, 0xF, true);
        hi = __builtin_amdgcn_mov_dpp((int)(bv >> 32), CTRL, 0xF, 0xF, true);
    } else {
        lo = __builtin_amdgcn_update_dpp((int)bf, (int)bv, CTRL, ROW_MASK, 0xF, false);
        hi = __builtin_amdgcn_update_dpp((int)(bf >> 32), (int)(bv >> 32), CTRL, ROW_MASK, 0xF, false);
    }
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// DPP move of a float; lanes without a source receive 0.0f (as dpp_f64).
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ float dpp_f32(float v)
{
    if constexpr (ROW_MASK == 0xF)
        return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xF, 0xF, true));
    else
        return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROW_MASK, 0xF, false));
}

// One reduction step: x <- x (*) (state moved by the DPP pattern); lanes
// without a source multiply by the identity.
template <int K, int CTRL, int ROW_MASK>
__device__ __forceinline__ void dpp_step(Acc& x, bool want_bound)
{
    Acc o;
#pragma unroll
    for (int k = 1; k <= K; ++k) o.a[k] = dpp_f64<CTRL, ROW_MASK>(x.a[k], 0.0);
    if (want_bound) {
        o.m = dpp_f32<CTRL, ROW_MASK>(x.m);
        o.eps = dpp_f32<CTRL, ROW_MASK>(x.eps);
        o.lsabs = dpp_f32<CTRL, ROW_MASK>(x.lsabs);
    }
    o.ls = dpp_f64<CTRL, ROW_MASK>(x.ls, 0.0);
    merge<K>(x, o, want_bound);
}

// Segmented reduction of the lane states with DPP row shifts and row
// broadcasts (no LDS traffic): lanes form segments of 2^lw consecutive lanes
// (2^lw <= 64) and, after lw steps, the last lane of every segment holds
// the product of its segment.  This is an inclusive Hillis-Steele scan
// whose steps never reach past 2^lw - 1 lanes below, so a segment's last
// lane sees only its own segment; lanes without a source multiply by the
// identity.  The fixed step pattern makes the result deterministic.
template <int K>
__device__ __forceinline__ void wave_reduce_seg(Acc& x, int lw, bool want_bound)
{
    constexpr int ROW_SHR1 = 0x111, ROW_SHR2 = 0x112, ROW_SHR4 = 0x114, ROW_SHR8 = 0x118;
    constexpr int ROW_BCAST15 = 0x142, ROW_BCAST31 = 0x143;
    if (lw >= 1) dpp_step<K, ROW_SHR1, 0xF>(x, want_bound);
    if (lw >= 2) dpp_step<K, ROW_SHR2, 0xF>(x, want_bound);
    if (lw >= 3) dpp_step<K, ROW_SHR4, 0xF>(x, want_bound);
    if (lw >= 4) dpp_step<K, ROW_SHR8, 0xF>(x, want_bound);
    // lane 15 of each row now holds its row; row 1 takes row 0's total, row 3 row 2's
    if (lw >= 5) dpp_step<K, ROW_BCAST15, 0xA>(x, want_bound);
    if (lw >= 6) dpp_step<K, ROW_BCAST31, 0xC>(x, want_bound);
}

// Inclusive product scan of a truncated polynomial over the wave's 64 lanes
// (lane l ends with the product of lanes 0..l), by the DPP steps of
// wave_reduce_seg on plain polynomials; lanes without a source multiply by
// the identity.
template <int K, int CTRL, int ROW_MASK>
__device__ __forceinline__ void poly_dpp_step(double (&a)[MAXK + 1])
{
    double o[MAXK + 1];
    o[0] = 0.0;
#pragma unroll
    for (int k = 1; k <= K; ++k) o[k] = dpp_f64<CTRL, ROW_MASK>(a[k], 0.0);
    pmul<K>(a, o);
}

template <int K>
__device__ __forceinline__ void poly_scan_incl(double (&a)[MAXK + 1])
{
    poly_dpp_step<K, 0x111, 0xF>(a);
    poly_dpp_step<K, 0x112, 0xF>(a);
    poly_dpp_step<K, 0x114, 0xF>(a);
    poly_dpp_step<K, 0x118, 0xF>(a);
    poly_dpp_step<K, 0x142, 0xA>(a);
    poly_dpp_step<K, 0x143, 0xC>(a);
}

// Sum over the wave's 64 lanes, returned to every lane.
__device__ __forceinline__ double wave_sum64(double v)
{
    v += dpp_f64<0x111, 0xF>(v, 0.0);
    v += dpp_f64<0x112, 0xF>(v, 0.0);
    v += dpp_f64<0x114, 0xF>(v, 0.0);
    v += dpp_f64<0x118, 0xF>(v, 0.0);
    v += dpp_f64<0x142, 0xA>(v, 0.0);
    v += dpp_f64<0x143, 0xC>(v, 0.0);
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)b, 63), hi = __builtin_amdgcn_readlane((int)(b >> 32), 63);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

__device__ __forceinline__ double lane_double(double v, int src)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_ds_bpermute(src << 2, (int)b);
    const int hi = __builtin_amdgcn_ds_bpermute(src << 2, (int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

constexpr int ACC_WORDS = MAXK + 4;   // doubles per wave in LDS

template <int K>
__device__ __forceinline__ void acc_store(const Acc& x, double* s)
{
#pragma unroll
    for (int k = 1; k <= K; ++k) s[k - 1] = x.a[k];
    s[MAXK] = (double)x.m;
    s[MAXK + 1] = x.ls;
    s[MAXK + 2] = (double)x.lsabs;
    s[MAXK + 3] = (double)x.eps;
}

template <int K>
__device__ __forceinline__ void acc_load(Acc& x, const double* s)
{
#pragma unroll
    for (int k = 1; k <= K; ++k) x.a[k] = s[k - 1];
    x.m = (float)s[MAXK];
    x.ls = s[MAXK + 1];
    x.lsabs = (float)s[MAXK + 2];
    x.eps = (float)s[MAXK + 3];
}

// Upper bound on every |[z^b] prod_{t in T} delta_t| (any subset T) summed
// over b <= K.  With M(z) = sum_t sum_e |delta_t[e]| z^e the product of the
// absolute-value polynomials is at most exp(M(z)) coefficient-wise
// (1 + x <= exp(x) for non-negative coefficients); M(z)^j starts at degree
// j and its coefficients sum to m^j (m = M(1)), so the sum over b <= K is at
// most T_K(m) = sum_{j <= K} m^j / j!, far below exp(m) once m exceeds K.
// Horner in FP32 over non-negative terms (a short chain at the end of every
// wave): m is rounded up on its conversion (the product by 1 + 2^-22 covers
// the conversion's and its own rounding, 2^-24 each), each of the K levels rounds the reciprocal 1/j,
// the product and the FMA once (at most 3K units of 2^-24 relative in all),
// covered by the factor 1 + 4 (K + 1) 2^-24; m is given as an upper bound;
// an overflow gives +inf.
template <int K>
__device__ __forceinline__ double abs_product_bound(double m)
{
    const float mf = (float)m * (1.0f + 2.384185791015625e-07f);
    float r = 1.0f;
#pragma unroll
    for (int j = K; j >= 1; --j) r = fmaf(mf * (1.0f / (float)j), r, 1.0f);
    return (double)r * (1.0 + (double)(4 * (K + 1)) * 5.9604644775390625e-08);
}

// ------------------------------------------------------------ read-out
// Q = A * (1 + sum_k a_k) with the affine partial sum giving A, and the
// a-priori bound on |Q - exact Smolyak value| from rounding.
template <int PREC, int K, int FAM>
__device__ void readout(const Acc& x, int d, int out_index, const double* __restrict__ prm, int rl_pairs,
                        int depth, double* out, double* bound)
{
    const bool want_bound = bound != nullptr;
    double s = 0.0;
#pragma unroll
    for (int k = K; k >= 1; --k) s += x.a[k];
    s += 1.0;
    // the bound's FP32 sums (each term rounded once to FP32, then added:
    // at most 2 (d + depth) roundings) raised to upper bounds
    const double marg = bound_sum_margin(d + depth + 4);
    const double m_up = (double)x.m * marg, eps_up = (double)x.eps * marg, lsabs_up = (double)x.lsabs * marg;
    const double sabs = want_bound ? abs_product_bound<K>(m_up) : 0.0;
    const double u64 = 1.1102230246251565e-16;
    // rounding of the affine sum: d - 1 additions, plus up to 3 roundings
    // per term where a term is not exact (product-peak log D, gaussian c hv^2)
    const double ls_err =
        u64 * (double)(FAM == FAM_EXP || FAM == FAM_OSC ? d : d + 3) * lsabs_up;
    // relative error of one surplus term: pair value (8 roundings) plus the
    // within-rule sum (FP64: a plain FMA chain over at most rl_pairs terms;
    // FP32 compensated: the FMA chain of the term's block, at most
    // kSumBlock roundings, blocks joined exactly; FP32 values with FP64
    // sums: the FP32 value's error, the FP64 chain adding a negligible
    // rl_pairs * 2^-53)
    const double rel = PREC == SG_PREC_FP64 ? u64 * (8.0 + (double)rl_pairs)
                       : PREC == SG_PREC_FP32_COMPENSATED
                           ? 5.9604644775390625e-08 * (9.0 + kSumBlock) + u64 * (double)rl_pairs
                           : 5.9604644775390625e-08 * 10.0 + u64 * (double)rl_pairs;
    // products of the sweep: (K+2) roundings per level of the product tree
    // (depth: the caller's bound on the tree depth)
    const double levels = (double)depth;
    double Q;
    if constexpr (FAM == FAM_OSC) {
        const double phase = 2.0 * 3.141592653589793 * prm[0] + x.ls;
        Q = cos(phase) * s;
        if (want_bound) {
            const double dsum = sabs * (rel * eps_up + (K + 2) * levels * u64);
            bound[out_index] = dsum + fabs(s) * (ls_err + u64 * (fabs(phase) + 4.0)) + fabs(Q) * 4.0 * u64;
        }
    } else {
        const double A = exp(FAM == FAM_PEAK ? -x.ls : x.ls);
        Q = A * s;
        if (want_bound) {
            const double dsum = sabs * (rel * eps_up + (K + 2) * levels * u64);
            bound[out_index] = A * dsum + fabs(Q) * (ls_err + 4.0 * u64 + u64 * fabs(x.ls));
        }
    }
    out[out_index] = Q;
}

// Number of node pairs of a (class, K) table (for the bound's sum length).
template <int RC, int K>
constexpr int total_pairs()
{
    int n = 0;
    for (int L = 2; L <= K + 1; ++L) n += rc_pairs(RC, L);
    return n;
}

// ----------------------------------------------------------- wave sweep
// Per-coordinate inputs of a family: the raw parameters (loaded one
// coordinate ahead of their use), then the pair-function parameters and the
// coordinate's term of the affine partial sum (log-amplitude or phase).
struct RawParam {
    double a, b;
};

template <int FAM>
__device__ __forceinline__ RawParam load_param(const double* __restrict__ prm, int d, int t)
{
    RawParam r;
    if constexpr (FAM == FAM_EXP) {
        r.a = prm[t];
        r.b = 0.0;
    } else if constexpr (FAM == FAM_OSC) {
        r.a = prm[1 + t];
        r.b = 0.0;
    } else {
        r.a = prm[t];
        r.b = prm[d + t];
    }
    return r;
}

template <int FAM>
__device__ __forceinline__ double coord_param(const RawParam& r, CoordParam& cp)
{
    if constexpr (FAM == FAM_EXP || FAM == FAM_OSC) {
        cp.p0 = r.a;
        cp.p1 = 0.0;
        return 0.5 * cp.p0;                       // exp: log g_t(1/2) = c_t/2; osc: phase a_t/2
    } else if constexpr (FAM == FAM_GAUSS) {
        const double hv = 0.5 - r.b;
        cp.p0 = r.a;
        cp.p1 = r.a * (2.0 * hv);                 // c (1 - 2u)
        return r.a * (hv * hv);                   // log g_t(1/2) = c (1/2 - u)^2
    } else {
        cp.p0 = 1.0 / (r.a * r.a);                // beta = b^-2
        cp.p1 = 0.5 - r.b;
        return log(fma(cp.p1, cp.p1, cp.p0));     // log D_t(1/2) = -log g_t(1/2)
    }
}

// One forward wave: its class and shape (wave-uniform) and this lane's
// problem, resolved from the descriptor before the sweep starts.
struct WaveInfo {
    int lw, rank, group, nprob;
    const double* r64;     // the class's record table (table-driven path)
    const float* r32;
    int d;                 // this lane's problem: dimension (0: idle lane),
    int out_index;         // its slot in out / bound,
    int64_t param_offset;  // its parameters in the caller's array
};

// Depth of the product tree behind one result: a lane's sequential chain of
// ceil(d / (2^lw * group)) coordinates, lw DPP levels, up to 3 group merges.
__device__ __forceinline__ int tree_depth(int d, int lw, int group)
{
    const int span = (1 << lw) * group;
    return (d + span - 1) / span + lw + 4;
}

// One wave sweeps its problems: lane l works on problem seg[l >> lw] and
// its coordinates t = rank*2^lw + (l & (2^lw - 1)) + j * 2^lw * group, then
// the segments are reduced and every segment's last lane reads out (group of
// one wave) or, for a multi-wave problem, leaves the wave's state in LDS for
// the group leader.  The next coordinate's parameters are loaded before the
// current coordinate is evaluated, so their latency overlaps the arithmetic
// (loading every coordinate's parameters up front instead makes all waves
// fetch the whole batch at once and wait for it before computing).
template <int PREC, int K, int RULE, int FAM>
__device__ __forceinline__ void wave_sweep(const WaveInfo& wi, const double* __restrict__ params, double* out,
                                           double* bound, double* lds_slot)
{
    constexpr int RC = rule_class_of(RULE);
    const bool want_bound = bound != nullptr;
    const int lane = threadIdx.x & 63;
    const int W = 1 << wi.lw;
    const int lis = lane & (W - 1);
    const int d = wi.d, out_index = wi.out_index;
    const double* __restrict__ prm = params + wi.param_offset;

    Acc x;
    acc_identity<K>(x);
    const int stride = W * wi.group;
    int t = wi.rank * W + lis;
    RawParam nxt{0.0, 0.0};
    if (t < d) nxt = load_param<FAM>(prm, d, t);
    while (t < d) {
        const RawParam cur = nxt;
        const int tn = t + stride;
        if (tn < d) nxt = load_param<FAM>(prm, d, tn);
        CoordParam cp;
        const double lterm = coord_param<FAM>(cur, cp);
        double del[MAXK + 1];
        double eps_t = 0.0;
        bool done = false;
        if constexpr (K <= KCONST && FAM != FAM_GAUSS) {
            if (FAM == FAM_PEAK || fabs(cp.p0) <= 2.0) {
                if constexpr (PREC == SG_PREC_FP64) surplus64_const<RULE, K, FAM>(cp, del, eps_t);
                else if constexpr (PREC == SG_PREC_FP32_COMPENSATED) surplus32_const<RULE, K, FAM>(cp, del, eps_t);
                else surplus32e_const<RULE, K, FAM>(cp, del, eps_t);
                done = true;
            }
        }
        if (!done) {
            // table-driven path: large parameters (any K) and K > KCONST.
            // The table addresses are loop-invariant; hiding them from the
            // optimiser keeps the table in scalar loads issued per coordinate
            // instead of hoisting hundreds of values into vector registers.
            int opaque = 0;
            asm volatile("" : "+s"(opaque));
            // (FP32 node values with FP64 sums fall back to FP64 values here)
            if constexpr (PREC != SG_PREC_FP32_COMPENSATED) surplus64<K, RC, FAM>(wi.r64 + opaque, cp, true, del, eps_t);
            else surplus32<K, RC, FAM>(wi.r64 + opaque, wi.r32 + opaque, cp, true, del, eps_t);
        }
        pmul<K>(x.a, del);
        if (want_bound) {
            double mt = 0.0;
#pragma unroll
            for (int k = 1; k <= K; ++k) mt += fabs(del[k]);
            x.m += (float)mt;
            x.eps += (float)eps_t;
            x.lsabs += (float)fabs(lterm);
        }
        x.ls += lterm;
        t = tn;
    }
    wave_reduce_seg<K>(x, wi.lw, want_bound);
    if (lis != W - 1) return;
    if (wi.group == 1) {
        if (out_index >= 0)
        {
            constexpr int np = total_pairs<RC, K>();
            readout<PREC, K, FAM>(x, d, out_index, prm, np, tree_depth(d, wi.lw, 1), out, bound);
        }
    } else {
        acc_store<K>(x, lds_slot);
    }
}

template <int PREC, int K, bool GAUSS>
__device__ __forceinline__ void wave_dispatch_k(int rule, int family, const WaveInfo& wi, const double* params,
                                                double* out, double* bound, double* lds_slot)
{
#define SG_WAVE(RULE, FAM) wave_sweep<PREC, K, RULE, FAM>(wi, params, out, bound, lds_slot)
#define SG_FAMS(RULE)                                         \
    do {                                                      \
        if (GAUSS && family == FAM_GAUSS) {                   \
            if constexpr (GAUSS) SG_WAVE(RULE, FAM_GAUSS);    \
        } else if (family == FAM_EXP) SG_WAVE(RULE, FAM_EXP); \
        else if (family == FAM_OSC) SG_WAVE(RULE, FAM_OSC);   \
        else SG_WAVE(RULE, FAM_PEAK);                         \
    } while (0)
    if constexpr (K <= KCONST) {
        // compiled tables differ per rule
        if (rule == SG_RULE_CLENSHAW_CURTIS) SG_FAMS(SG_RULE_CLENSHAW_CURTIS);
        else if (rule == SG_RULE_TRAPEZOID) SG_FAMS(SG_RULE_TRAPEZOID);
        else if (rule == SG_RULE_GAUSS_LEGENDRE) SG_FAMS(SG_RULE_GAUSS_LEGENDRE);
        else if (rule == SG_RULE_GAUSS_PATTERSON) SG_FAMS(SG_RULE_GAUSS_PATTERSON);
        else SG_FAMS(SG_RULE_GAUSS_LEGENDRE_PAPER);
    } else {
        // table-driven only: one instantiation per structure class
        const int rc = rule_class_of(rule);
        if (rc == RC_NESTED) SG_FAMS(SG_RULE_CLENSHAW_CURTIS);
        else if (rc == RC_GL2) SG_FAMS(SG_RULE_GAUSS_LEGENDRE);
        else if (rc == RC_GP) SG_FAMS(SG_RULE_GAUSS_PATTERSON);
        else SG_FAMS(SG_RULE_GAUSS_LEGENDRE_PAPER);
    }
#undef SG_FAMS
#undef SG_WAVE
}

// Group leader: merge the group's wave states in wave order, read out.
template <int PREC, int K, bool GAUSS>
__device__ __forceinline__ void group_finish_k(int rule, int family, int group, const FwdSeg& lp,
                                               const double* lds_first, const double* params, double* out,
                                               double* bound)
{
    const bool want_bound = bound != nullptr;
    Acc x, y;
    acc_identity<K>(x);
    acc_identity<K>(y);
    acc_load<K>(x, lds_first);
    for (int g = 1; g < group; ++g) {
        acc_load<K>(y, lds_first + g * ACC_WORDS);
        merge<K>(x, y, want_bound);
    }
    const double* prm = params + lp.param_offset;
    const int rc = rule_class_of(rule);
    constexpr int np_nested = total_pairs<RC_NESTED, K>(), np_gl2 = total_pairs<RC_GL2, K>(),
                  np_gp = total_pairs<RC_GP, K>(), np_glp = total_pairs<RC_GLP, K>();
    const int np = rc == RC_NESTED ? np_nested : rc == RC_GL2 ? np_gl2 : rc == RC_GP ? np_gp : np_glp;
    const int depth = tree_depth(lp.d, 6, group);
    if constexpr (GAUSS) {
        if (family == FAM_GAUSS) {
            readout<PREC, K, FAM_GAUSS>(x, lp.d, lp.out_index, prm, np, depth, out, bound);
            return;
        }
    }
    if (family == FAM_EXP) readout<PREC, K, FAM_EXP>(x, lp.d, lp.out_index, prm, np, depth, out, bound);
    else if (family == FAM_OSC) readout<PREC, K, FAM_OSC>(x, lp.d, lp.out_index, prm, np, depth, out, bound);
    else readout<PREC, K, FAM_PEAK>(x, lp.d, lp.out_index, prm, np, depth, out, bound);
}

// Flat dispatch of a forward wave to its class's code: one switch on a
// class index.  (Nested run-time tests of K, then rule, then family make a
// failing test jump over a whole class body to the next test, so a wave
// crosses up to a dozen cold instruction-cache lines before its first
// useful instruction.)  The compiled-table path (K <= KCONST) has code per
// rule; the table-driven path per structure class, under the class's
// representative rule.
__host__ __device__ __forceinline__ constexpr int fam_slot(int family)
{
    return family == FAM_EXP ? 0 : family == FAM_OSC ? 1 : family == FAM_PEAK ? 2 : 3;
}
__host__ __device__ __forceinline__ constexpr int representative_rule(int rule)
{
    return rule_class_of(rule) == RC_NESTED ? SG_RULE_CLENSHAW_CURTIS
           : rule_class_of(rule) == RC_GL2  ? SG_RULE_GAUSS_LEGENDRE
           : rule_class_of(rule) == RC_GP   ? SG_RULE_GAUSS_PATTERSON
                                            : SG_RULE_GAUSS_LEGENDRE_PAPER;
}
__host__ __device__ constexpr int class_slot(int K, int rule, int fslot) { return (K * 8 + rule) * 4 + fslot; }
__host__ __device__ __forceinline__ constexpr int class_index(int K, int rule, int family)
{
    return class_slot(K, K <= KCONST ? rule : representative_rule(rule), fam_slot(family));
}

template <int PREC, int KMAXP, bool GAUSS, int K, int R, int F>
__device__ __forceinline__ void wave_case(const WaveInfo& wi, const double* params, double* out, double* bound,
                                          double* lds_slot)
{
    constexpr int FAM = F == 0 ? FAM_EXP : F == 1 ? FAM_OSC : F == 2 ? FAM_PEAK : FAM_GAUSS;
    if constexpr (K <= KMAXP && (GAUSS || FAM != FAM_GAUSS) && (K <= KCONST || R == representative_rule(R)))
        wave_sweep<PREC, K, R, FAM>(wi, params, out, bound, lds_slot);
}

template <int PREC, int KMAXP, bool GAUSS>
__device__ __forceinline__ void wave_switch(int cls, const WaveInfo& wi, const double* params, double* out,
                                            double* bound, double* lds_slot)
{
    static_assert(KMAXP <= 8, "class index covers K <= 8");
    switch (cls) {
#define SG_C(K, R, F)                                                                   \
    case class_slot(K, R, F):                                                           \
        wave_case<PREC, KMAXP, GAUSS, K, R, F>(wi, params, out, bound, lds_slot);         \
        break;
#define SG_CR(K, R) SG_C(K, R, 0) SG_C(K, R, 1) SG_C(K, R, 2) SG_C(K, R, 3)
#define SG_CK(K) SG_CR(K, 1) SG_CR(K, 2) SG_CR(K, 3) SG_CR(K, 4) SG_CR(K, 5)
        SG_CK(0) SG_CK(1) SG_CK(2) SG_CK(3) SG_CK(4) SG_CK(5) SG_CK(6) SG_CK(7) SG_CK(8)
#undef SG_CK
#undef SG_CR
#undef SG_C
    default:
        break;
    }
}

// Dispatch a runtime K in [0, KMAXP] to a compile-time K.
template <int KMAXP, class F>
__device__ __forceinline__ void switch_k(int K, F&& f)
{
    static_for<0, KMAXP + 1>([&](auto kc) {
        if (K == decltype(kc)::value) f(kc);
    });
}

// One workgroup descriptor: 4 waves; wave w runs wg->w[w].  A problem
// spanning several waves sits in consecutive waves of the workgroup and is
// merged through LDS by its first wave.  Every thread of the workgroup must
// call this (it may synchronise the workgroup).
// A 32-bit value from another lane of the wave (ds_bpermute).
__device__ __forceinline__ int lane_read(int v, int src_lane)
{
    return __builtin_amdgcn_ds_bpermute(src_lane << 2, v);
}

template <int PREC, int KMAXP, bool GAUSS>
__device__ __forceinline__ void run_workgroup(const FwdWG* wg, const double* __restrict__ pool64,
                                              const float* __restrict__ pool32, const double* __restrict__ params,
                                              double* __restrict__ out, double* __restrict__ bound, double* lds)
{
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // wave-uniform
    const FwdWave* wd = &wg->w[w];
    // lane i fetches segment record i mod kWaveProbs together with the
    // wave's scalars (no dependence between the two loads); each lane then
    // takes its own segment's record from the lane that holds it
    const int lane = threadIdx.x & 63;
    const FwdSeg cand = wd->seg[lane & (kWaveProbs - 1)];
    const int K = __builtin_amdgcn_readfirstlane(wd->K);
    const int rule = __builtin_amdgcn_readfirstlane(wd->rule);
    const int family = __builtin_amdgcn_readfirstlane(wd->family);
    WaveInfo wi;
    wi.lw = __builtin_amdgcn_readfirstlane(wd->lw);
    wi.rank = __builtin_amdgcn_readfirstlane(wd->rank);
    wi.group = __builtin_amdgcn_readfirstlane(wd->group);
    wi.nprob = __builtin_amdgcn_readfirstlane(wd->nprob);
    wi.r64 = pool64 + __builtin_amdgcn_readfirstlane(wd->off64);
    wi.r32 = pool32 + __builtin_amdgcn_readfirstlane(wd->off32);
    {
        const int sg = lane >> wi.lw;   // lw >= 2: sg < kWaveProbs
        const int d = lane_read(cand.d, sg);
        const int oi = lane_read(cand.out_index, sg);
        const unsigned int plo = (unsigned int)lane_read((int)(cand.param_offset & 0xffffffffll), sg);
        const int phi = lane_read((int)(cand.param_offset >> 32), sg);
        const bool live = sg < wi.nprob;
        wi.d = live ? d : 0;
        wi.out_index = live ? oi : -1;
        wi.param_offset = live ? (int64_t)(((uint64_t)(unsigned int)phi << 32) | plo) : 0;
    }
    const bool grouped = __builtin_amdgcn_readfirstlane(wg->w[0].grouped) != 0;
    if (wi.nprob > 0)
        wave_switch<PREC, KMAXP, GAUSS>(__builtin_amdgcn_readfirstlane(class_index(K, rule, family)), wi, params, out,
                                        bound, lds + w * ACC_WORDS);
    if (!grouped) return;
    __syncthreads();
    if (wi.nprob > 0 && wi.group > 1 && wi.rank == 0 && (threadIdx.x & 63) == 0) {
        const FwdSeg lp = wd->seg[0];
        switch_k<KMAXP>(K, [&](auto kc) {
            group_finish_k<PREC, decltype(kc)::value, GAUSS>(rule, family, wi.group, lp, lds + w * ACC_WORDS, params, out,
                                                      bound);
        });
    }
}

// Forward kernel.  queue == nullptr: hardware dispatch, workgroup b runs
// descriptor b.  Otherwise the persistent form: a grid of G workgroups
// sized to the resident capacity; workgroup b runs descriptor b first (no
// atomic: every workgroup asking the one counter at once serialises
// hundreds of atomics), then pops further descriptors (longest first) from
// the work queue, G + queue[0] being the next index, and leaves at its first
// index past the end.  A launch makes exactly nwg - G + G = nwg pops
// (numbered 0 .. nwg - 1 by the counter), so the pop numbered nwg - 1 is
// the last of all: no workgroup pops again, and that workgroup returns the
// counter to zero for the next launch on the stream, without a memset or
// an exit count (graph-safe).  With G >= nwg nothing is popped.  Launches
// of one queue must not overlap.
// GAUSS: the instantiation for plans that hold gaussian problems (it runs
// every family; kept apart so that the gaussian code does not weigh on the
// other plans' kernels).
template <int PREC, int KMAXP, bool GAUSS = false>
__global__ void __launch_bounds__(256)
k_forward(const FwdWG* __restrict__ wgs, int nwg, unsigned int* __restrict__ queue,
          const double* __restrict__ pool64, const float* __restrict__ pool32,
          const double* __restrict__ params, double* __restrict__ out, double* __restrict__ bound)
{
    __shared__ double lds[4 * ACC_WORDS];
    __shared__ int next;
    int idx = blockIdx.x;
    for (;;) {
        if (idx >= nwg) break;
        run_workgroup<PREC, KMAXP, GAUSS>(wgs + idx, pool64, pool32, params, out, bound, lds);
        if (!queue || (int)gridDim.x >= nwg) break;   // no descriptor beyond the static ones
        if (threadIdx.x == 0) {
            const unsigned int k = atomicAdd(&queue[0], 1u);
            if (k == (unsigned int)(nwg - 1)) atomicExch(&queue[0], 0u);   // the last pop of the launch
            next = (int)gridDim.x + (int)k;
        }
        __syncthreads();
        idx = __builtin_amdgcn_readfirstlane(next);
        __syncthreads();   // every thread has read `next` before it is overwritten
    }
}

// ================================================================ adjoint
// Reverse sweep.  With S(z) = prod_t delta_t(z) (monic, truncated at z^K)
// and s = sum_{b<=K} [z^b] S:
//   ds/d delta_t[e] = sum_{j=0}^{K-e} [z^j] R_t,   R_t = prod_{t' != t} delta_t',
// where R_t is formed from exclusive prefix and suffix products across the
// sweep (no division by delta_t), and
//   d delta_t[e] / d p_t = sum_p dW[e][p] ds_p/dp_t
// is a within-rule sum of derivative pair values.  The affine partial sum
// (log-amplitude or phase) contributes its own term.

// sinh(v)/v = sum z^k/(2k+1)!, sin(v)/v = sum (-z)^k/(2k+1)!, z = v^2.
__device__ __forceinline__ double series_s64(double z)
{
    double p = 1.0 / 355687428096000.0;                // 1/17!
    p = fma(p, z, 1.0 / 1307674368000.0);              // 1/15!
    p = fma(p, z, 1.0 / 6227020800.0);                 // 1/13!
    p = fma(p, z, 1.0 / 39916800.0);                   // 1/11!
    p = fma(p, z, 1.0 / 362880.0);                     // 1/9!
    p = fma(p, z, 1.0 / 5040.0);                       // 1/7!
    p = fma(p, z, 1.0 / 120.0);                        // 1/5!
    p = fma(p, z, 1.0 / 6.0);                          // 1/3!
    p = fma(p, z, 1.0);
    return p;
}

__device__ __forceinline__ float series_s32(float z)
{
    float p = 1.0f / 362880.0f;
    p = fmaf(p, z, 1.0f / 5040.0f);
    p = fmaf(p, z, 1.0f / 120.0f);
    p = fmaf(p, z, 1.0f / 6.0f);
    p = fmaf(p, z, 1.0f);
    return p;
}

// d s(y) / d parameter for exp-sum (d/dc: 2 y sinh(c y)) and oscillatory
// (d/da: -2 y sin(a y)).
template <int FAM>
__device__ __forceinline__ double dpair64(const CoordParam& cp, double y)
{
    const double v = cp.p0 * y;
    const double z = v * v;
    if (fabs(v) <= 0.5) return FAM == FAM_EXP ? 2.0 * y * v * series_s64(z) : -2.0 * y * v * series_s64(-z);
    return FAM == FAM_EXP ? 2.0 * y * sinh(v) : -2.0 * y * sin(v);
}

template <int FAM>
__device__ __forceinline__ float dpair32(const CoordParam& cp, double y)
{
    const float v = (float)(cp.p0 * y);
    const float yf = (float)y;
    const float z = v * v;
    if (fabsf(v) <= 0.5f) return FAM == FAM_EXP ? 2.0f * yf * v * series_s32(z) : -2.0f * yf * v * series_s32(-z);
    return FAM == FAM_EXP ? 2.0f * yf * sinhf(v) : -2.0f * yf * sinf(v);
}

// Product-peak: s = 2 y^2 N / (Dp Dm), N = 3 hv^2 - beta - y^2,
// Dp = beta + (y + hv)^2, Dm = beta + (y - hv)^2; derivatives in beta and hv.
__device__ __forceinline__ void dpair_peak64(const CoordParam& cp, double y, double& ds_dbeta, double& ds_dhv)
{
    const double beta = cp.p0, hv = cp.p1;
    const double y2 = y * y;
    const double dp = y + hv, dm = y - hv;
    const double Dp = fma(dp, dp, beta), Dm = fma(dm, dm, beta);
    const double D = Dp * Dm;
    const double N = fma(3.0 * hv, hv, -beta) - y2;
    const double iD2 = 1.0 / (D * D);
    // d(Dp Dm)/d beta = Dp + Dm;  d(Dp Dm)/d hv = 2 dp Dm - 2 dm Dp
    ds_dbeta = 2.0 * y2 * (-D - N * (Dp + Dm)) * iD2;
    ds_dhv = 2.0 * y2 * (6.0 * hv * D - N * (2.0 * dp * Dm - 2.0 * dm * Dp)) * iD2;
}

// Gaussian: s = 2 (e^{c y^2} cosh(c b y) - 1) with b = 1 - 2u; derivatives
// in c (at fixed u) and in u (db/du = -2).  The exponentials come from the
// branch-free expm1 of the forward pass (two per pair instead of the
// library's exp, cosh and sinh, which cost the kernel its registers):
// with F = expm1(|v|) >= 0, cosh v = 1 + F^2/(2(1 + F)) and
// |sinh v| = (F + F/(1 + F))/2, both free of cancellation.
__device__ __forceinline__ void dpair_gauss64(double c, double b, double y, double& ds_dc, double& ds_du)
{
    const double e = 1.0 + expm1_any(c * (y * y));
    const double v = c * (b * y);
    const double F = expm1_any(fabs(v));
    const double r = F / (1.0 + F);
    const double ch = fma(0.5 * F, r, 1.0);
    const double sh = copysign(0.5 * (F + r), v);
    ds_dc = 2.0 * e * fma(y * y, ch, b * y * sh);
    ds_du = -4.0 * c * y * e * sh;
}

// sum_e G[e] dS[e] and sum_e G[e] dT[e] for the two derivative surpluses dS,
// dT of one coordinate without forming them: each pair's weights are
// contracted with G first, then multiplied by its two derivative values
// (one evaluation per pair, and no surplus arrays held in registers).
template <int K, int RC, class PF>
__device__ __forceinline__ void contract_pairs2(const double* __restrict__ r64, const double (&G)[MAXK + 1],
                                                PF&& pf, double& sa, double& sb)
{
    sa = 0.0;
    sb = 0.0;
    static_for<2, K + 2>([&](auto Lc) {
        constexpr int L = decltype(Lc)::value;
        constexpr int np = rc_pairs(RC, L), lo = rc_elo(L), hi = rc_ehi(RC, K, L);
        constexpr int rl = rc_rec64(RC, K, L), off = rc_off64(RC, K, L);
#pragma unroll 2
        for (int j = 0; j < np; ++j) {
            const double* r = r64 + off + j * rl;
            double wg = 0.0;
#pragma unroll
            for (int e = lo; e <= hi; ++e) wg = fma(G[e], r[1 + e - lo], wg);
            double a, b;
            pf(r[0], a, b);
            sa = fma(wg, a, sa);
            sb = fma(wg, b, sb);
        }
    });
}

// Inclusive scans of monic truncated polynomials across the 64 lanes.
template <int K>
__device__ __forceinline__ void shfl_poly_up(double (&o)[MAXK + 1], const double (&x)[MAXK + 1], int off)
{
#pragma unroll
    for (int k = 1; k <= K; ++k) o[k] = __shfl_up(x[k], off);
}
template <int K>
__device__ __forceinline__ void shfl_poly_down(double (&o)[MAXK + 1], const double (&x)[MAXK + 1], int off)
{
#pragma unroll
    for (int k = 1; k <= K; ++k) o[k] = __shfl_down(x[k], off);
}
template <int K>
__device__ __forceinline__ void poly_one(double (&x)[MAXK + 1])
{
#pragma unroll
    for (int k = 0; k <= MAXK; ++k) x[k] = 0.0;
}

constexpr int ADJ_WORDS = MAXK + 2;   // doubles per wave in LDS: wave product + affine sum

template <int PREC, int K, int RULE, int FAM>
__device__ __forceinline__ void wave_adjoint(const ProbDev& P, int rank, int group, bool grouped,
                                             const double* pool64, const float* pool32,
                                             const double* __restrict__ params, const double* __restrict__ gout,
                                             double* __restrict__ grad, double* __restrict__ ws, double* lds)
{
    constexpr int RC = rule_class_of(RULE);
    // the compiled-table surpluses (series forms, |parameter| <= 2)
    constexpr bool kConst = K <= KCONST && (FAM == FAM_EXP || FAM == FAM_OSC);
    const int lane = threadIdx.x & 63;
    const int d = P.d;
    const double* __restrict__ r64 = pool64 + P.off64;
    const float* __restrict__ r32 = pool32 + P.off32;
    const double* __restrict__ prm = params + P.param_offset;
    double* __restrict__ wsp = ws + P.ws_off;
    const int stride = 64 * group;
    // at most one coordinate per lane: its surpluses stay in registers and
    // the workspace is not touched
    const bool single = d <= stride;

    auto coord_param = [&](int t, CoordParam& cp) -> double {
        if constexpr (FAM == FAM_EXP) {
            cp.p0 = prm[t];
            cp.p1 = 0.0;
            return 0.5 * cp.p0;
        } else if constexpr (FAM == FAM_OSC) {
            cp.p0 = prm[1 + t];
            cp.p1 = 0.0;
            return 0.5 * cp.p0;
        } else if constexpr (FAM == FAM_GAUSS) {
            const double c = prm[t], hv = 0.5 - prm[d + t];
            cp.p0 = c;
            cp.p1 = c * (2.0 * hv);
            return c * (hv * hv);                  // log g_t(1/2)
        } else {
            const double b = prm[t], u = prm[d + t];
            cp.p0 = 1.0 / (b * b);
            cp.p1 = 0.5 - u;
            return log(fma(cp.p1, cp.p1, cp.p0));
        }
    };

    // pass 1: surpluses of this lane's coordinates (in the workspace unless
    // single), the lane's product and affine sum
    double L[MAXK + 1];
    poly_one<K>(L);
    double own[MAXK + 1];
    poly_one<K>(own);
    double ls = 0.0;
    for (int t = rank * 64 + lane; t < d; t += stride) {
        CoordParam cp;
        ls += coord_param(t, cp);
        double del[MAXK + 1], eps = 0.0;
        bool done = false;
        if constexpr (kConst) {
            if (fabs(cp.p0) <= 2.0) {
                if constexpr (PREC == SG_PREC_FP64) surplus64_const<RULE, K, FAM>(cp, del, eps);
                else surplus32_const<RULE, K, FAM>(cp, del, eps);
                done = true;
            }
        }
        if (!done) {
            int opaque = 0;
            asm volatile("" : "+s"(opaque));
            if constexpr (PREC == SG_PREC_FP64) surplus64<K, RC, FAM>(r64 + opaque, cp, false, del, eps);
            else surplus32<K, RC, FAM>(r64 + opaque, r32 + opaque, cp, false, del, eps);
        }
        if (single) {
#pragma unroll
            for (int k = 1; k <= K; ++k) own[k] = del[k];
        } else {
#pragma unroll
            for (int k = 1; k <= K; ++k) wsp[(size_t)t * K + (k - 1)] = del[k];
        }
        pmul<K>(L, del);
    }

    // exclusive prefix and suffix products across the wave's lanes: DPP
    // scans, the suffix as the prefix scan of the lanes in reverse order
    double pre[MAXK + 1], suf[MAXK + 1];
#pragma unroll
    for (int k = 0; k <= MAXK; ++k) { pre[k] = L[k]; suf[k] = 0.0; }
#pragma unroll
    for (int k = 1; k <= K; ++k) suf[k] = lane_double(L[k], 63 - lane);
    poly_scan_incl<K>(pre);
    poly_scan_incl<K>(suf);
    double wave_tot[MAXK + 1];
    wave_tot[0] = 0.0;
#pragma unroll
    for (int k = 1; k <= K; ++k) {
        const long long bits = __double_as_longlong(pre[k]);
        const int lo = __builtin_amdgcn_readlane((int)bits, 63), hi = __builtin_amdgcn_readlane((int)(bits >> 32), 63);
        wave_tot[k] = __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
    }
    {
        double tmp[MAXK + 1];
#pragma unroll
        for (int k = 1; k <= K; ++k) {
            tmp[k] = dpp_f64<0x138, 0xF>(pre[k], 0.0);          // wave_shr:1, lane 0 gets the identity
            suf[k] = lane_double(suf[k], lane == 63 ? 0 : 62 - lane);
        }
#pragma unroll
        for (int k = 1; k <= K; ++k) {
            pre[k] = tmp[k];
            if (lane == 63) suf[k] = 0.0;
        }
    }
    ls = wave_sum64(ls);

    // across the waves of the group: wave products in rank order
    double total[MAXK + 1];
#pragma unroll
    for (int k = 0; k <= MAXK; ++k) total[k] = wave_tot[k];
    if (grouped) {
        if (lane == 0) {
#pragma unroll
            for (int k = 1; k <= K; ++k) lds[k - 1] = wave_tot[k];
            lds[MAXK] = ls;
        }
        __syncthreads();
        if (group > 1) {
            const double* base = lds - rank * ADJ_WORDS;
            double wp[MAXK + 1], ws_[MAXK + 1], o[MAXK + 1];
            poly_one<K>(wp);
            poly_one<K>(ws_);
            poly_one<K>(o);
            double lsum = 0.0;
            for (int r = 0; r < group; ++r) {
#pragma unroll
                for (int k = 1; k <= K; ++k) o[k] = base[r * ADJ_WORDS + k - 1];
                lsum += base[r * ADJ_WORDS + MAXK];
                if (r < rank) pmul<K>(wp, o);
                if (r > rank) pmul<K>(ws_, o);
            }
            pmul<K>(pre, wp);
            pmul<K>(suf, ws_);
#pragma unroll
            for (int k = 1; k <= K; ++k) total[k] = wave_tot[k];
            pmul<K>(total, wp);
            pmul<K>(total, ws_);
            ls = lsum;
        }
    }

    // read-out quantities
    double s = 1.0;
#pragma unroll
    for (int k = K; k >= 1; --k) s += total[k];
    const double g = gout[P.out_index];
    double A = 1.0, cph = 0.0, sph = 0.0;
    if constexpr (FAM == FAM_OSC) {
        const double phase = 2.0 * 3.141592653589793 * prm[0] + ls;
        sincos(phase, &sph, &cph);
        if (rank == 0 && lane == 0) grad[P.param_offset] = g * (-2.0 * 3.141592653589793 * sph * s);
    } else {
        A = exp(FAM == FAM_PEAK ? -ls : ls);
    }

    // pass 2: per coordinate, R_t from prefix, suffix and the lane's other
    // coordinates; then the contraction with the derivative surpluses
    for (int t = rank * 64 + lane; t < d; t += stride) {
        double R[MAXK + 1];
#pragma unroll
        for (int k = 0; k <= MAXK; ++k) R[k] = pre[k];
        pmul<K>(R, suf);
        if (!single) {
            for (int t2 = rank * 64 + lane; t2 < d; t2 += stride) {
                if (t2 == t) continue;
                double o[MAXK + 1];
                o[0] = 1.0;
#pragma unroll
                for (int k = 1; k <= K; ++k) o[k] = wsp[(size_t)t2 * K + (k - 1)];
                pmul<K>(R, o);
            }
        }
        // G[e] = sum_{j <= K-e} R[j], R[0] = 1
        double G[MAXK + 1];
        {
            double c = 1.0;
            G[K] = 1.0;
#pragma unroll
            for (int e = K - 1; e >= 1; --e) { c += R[K - e]; G[e] = c; }
        }
        CoordParam cp;
        coord_param(t, cp);
        if constexpr (FAM == FAM_GAUSS) {
            int opaque = 0;
            asm volatile("" : "+s"(opaque));
            const double c = prm[t], hv = 0.5 - prm[d + t], b = 2.0 * hv;
            double dsc, dsu;
            contract_pairs2<K, RC>(r64 + opaque, G,
                                   [&](double y, double& a, double& e) { dpair_gauss64(c, b, y, a, e); }, dsc, dsu);
            // Q = A s, A = prod exp(c_t hv_t^2): dA/dc_t = hv_t^2 A, dA/du_t = -2 c_t hv_t A
            grad[P.param_offset + t] = g * A * fma(s, hv * hv, dsc);
            grad[P.param_offset + d + t] = g * A * fma(s, -2.0 * c * hv, dsu);
        } else if constexpr (FAM == FAM_PEAK) {
            int opaque = 0;
            asm volatile("" : "+s"(opaque));
            double db[MAXK + 1], du[MAXK + 1], eps = 0.0;
            surplus64g<K, RC>(r64 + opaque, [&](double y) { double a, b; dpair_peak64(cp, y, a, b); return a; },
                              false, db, eps);
            surplus64g<K, RC>(r64 + opaque, [&](double y) { double a, b; dpair_peak64(cp, y, a, b); return b; },
                              false, du, eps);
            double dsb = 0.0, dsh = 0.0;
#pragma unroll
            for (int e = 1; e <= K; ++e) { dsb = fma(G[e], db[e], dsb); dsh = fma(G[e], du[e], dsh); }
            const double b = prm[t];
            const double dbeta_db = -2.0 / (b * b * b);
            const double Dc = fma(cp.p1, cp.p1, cp.p0);            // D_t(1/2)
            // Q = A s, A = prod 1/D_t(1/2): dA/dbeta = -A/Dc, dA/dhv = -2 hv A/Dc
            const double dQ_dbeta = A * dsb - A * s / Dc;
            const double dQ_dhv = A * dsh - 2.0 * cp.p1 * A * s / Dc;
            grad[P.param_offset + t] = g * dQ_dbeta * dbeta_db;
            grad[P.param_offset + d + t] = g * (-dQ_dhv);         // hv = 1/2 - u
        } else {
            double dd[MAXK + 1];
            bool done = false;
            if constexpr (kConst) {
                if (fabs(cp.p0) <= 2.0) {
                    if constexpr (PREC == SG_PREC_FP64) dsurplus64_const<RULE, K, FAM>(cp, dd);
                    else dsurplus32_const<RULE, K, FAM>(cp, dd);
                    done = true;
                }
            }
            if (!done) {
                int opaque = 0;
                asm volatile("" : "+s"(opaque));
                double eps = 0.0;
                if constexpr (PREC == SG_PREC_FP64)
                    surplus64g<K, RC>(r64 + opaque, [&](double y) { return dpair64<FAM>(cp, y); }, false, dd, eps);
                else
                    surplus32g<K, RC>(r64 + opaque, r32 + opaque, [&](double y) { return dpair32<FAM>(cp, y); },
                                      false, dd, eps);
            }
            double ds = 0.0;
#pragma unroll
            for (int e = 1; e <= K; ++e) ds = fma(G[e], dd[e], ds);
            if constexpr (FAM == FAM_EXP) {
                grad[P.param_offset + t] = g * A * (ds + 0.5 * s);             // dA/dc_t = A/2
            } else {
                grad[P.param_offset + 1 + t] = g * (cph * ds - 0.5 * sph * s); // d phase/d a_t = 1/2
            }
        }
    }
}

// Flat dispatch of a reverse-sweep wave (the forward's class index).
template <int PREC, bool GAUSS, int K, int R, int F>
__device__ __forceinline__ void adjoint_case(const ProbDev& P, int rank, int group, bool grouped, const double* pool64,
                                             const float* pool32, const double* params, const double* gout,
                                             double* grad, double* ws, double* lds)
{
    constexpr int FAM = F == 0 ? FAM_EXP : F == 1 ? FAM_OSC : F == 2 ? FAM_PEAK : FAM_GAUSS;
    if constexpr ((GAUSS || FAM != FAM_GAUSS) && (K <= KCONST || R == representative_rule(R)))
        wave_adjoint<PREC, K, R, FAM>(P, rank, group, grouped, pool64, pool32, params, gout, grad, ws, lds);
}

template <int PREC, bool GAUSS>
__device__ __forceinline__ void adjoint_switch(int cls, const ProbDev& P, int rank, int group, bool grouped,
                                               const double* pool64, const float* pool32, const double* params,
                                               const double* gout, double* grad, double* ws, double* lds)
{
    switch (cls) {
#define SG_C(K, R, F)                                                                                   \
    case class_slot(K, R, F):                                                                           \
        adjoint_case<PREC, GAUSS, K, R, F>(P, rank, group, grouped, pool64, pool32, params, gout, grad, ws, lds); \
        break;
#define SG_CR(K, R) SG_C(K, R, 0) SG_C(K, R, 1) SG_C(K, R, 2) SG_C(K, R, 3)
#define SG_CK(K) SG_CR(K, 1) SG_CR(K, 2) SG_CR(K, 3) SG_CR(K, 4) SG_CR(K, 5)
        SG_CK(0) SG_CK(1) SG_CK(2) SG_CK(3) SG_CK(4) SG_CK(5) SG_CK(6) SG_CK(7) SG_CK(8)
#undef SG_CK
#undef SG_CR
#undef SG_C
    default:
        break;
    }
}

template <int PREC, bool GAUSS = false>
__global__ void __launch_bounds__(256)
k_adjoint(const WGDesc* __restrict__ wgs, const ProbDev* __restrict__ probs, const double* __restrict__ pool64,
          const float* __restrict__ pool32, const double* __restrict__ params, const double* __restrict__ gout,
          double* __restrict__ grad, double* __restrict__ ws)
{
    __shared__ double lds[4 * ADJ_WORDS];
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const WGDesc* desc = wgs + blockIdx.x;
    struct { int32_t prob; int16_t rank, group; } sl;
    sl.prob = __builtin_amdgcn_readfirstlane(desc->slot[w].prob);
    sl.rank = (int16_t)__builtin_amdgcn_readfirstlane(desc->slot[w].rank);
    sl.group = (int16_t)__builtin_amdgcn_readfirstlane(desc->slot[w].group);
    // the four group sizes read together (no short-circuit chain of loads)
    const int g0 = __builtin_amdgcn_readfirstlane(desc->slot[0].group);
    const int g1 = __builtin_amdgcn_readfirstlane(desc->slot[1].group);
    const int g2 = __builtin_amdgcn_readfirstlane(desc->slot[2].group);
    const int g3 = __builtin_amdgcn_readfirstlane(desc->slot[3].group);
    const bool grouped = ((g0 > 1) | (g1 > 1) | (g2 > 1) | (g3 > 1)) != 0;
    if (sl.prob < 0) {
        if (grouped) __syncthreads();
        return;
    }
    const ProbDev P = desc->slot[w].p;
    const int cls = __builtin_amdgcn_readfirstlane(class_index(P.K, P.rule, P.family));
    adjoint_switch<PREC, GAUSS>(cls, P, sl.rank, sl.group, grouped, pool64, pool32, params, gout, grad, ws,
                                lds + w * ADJ_WORDS);
}

}  // namespace dev
}  // namespace sg
