// Literal point-by-point evaluation of the Smolyak sum (2.6)-(2.7) on the
// GPU: the general path, valid for integrands that do not factor per
// coordinate, and an independent check of the factorised sweep.
//
// Q = f(c) + sum_{l in window} coef(|l|) sum_{points x of the tensor rule of l}
//            w(x) (f(x) - f(c)),
// with c the centre, coef(|l|) = (-1)^(q-|l|) C(d-1, q-|l|), and the
// centring valid because every tensor rule's weights sum to 1 and the
// coefficients sum to 1 over the window.
//
// Work split: the window's multi-indices in canonical order (excess
// ascending, then (l_1..l_d) decreasing lexicographically) are cut into
// chunks of 64 ranks, dealt round-robin to the waves of the grid.  The lanes
// of a wave unrank the 64 ranks of a chunk in parallel (into LDS); the wave
// then walks the chunk's multi-indices.  For each one it stages its
// "frontier" in LDS: for every active coordinate (level >= 2) and every node
// of that coordinate's level, the node weight and the node's contribution to
// the clustered partial quantity (the affine partial sum a_i (x - 1/2) of a
// ridge integrand, or log(g_i(x)/g_i(1/2)) of a product integrand).  The
// active coordinates are then split into two groups (the split that
// minimises the sum of the two groups' tensor sizes, at most 258 for K <= 8)
// and each group's tensor of partial sums, weight products and magnitude
// sums is staged too, so a point costs two LDS entries whatever its number
// of active coordinates.  Lanes cover the tensor points; f(x) - f(c) is
// formed without cancellation from the partial quantity (short Taylor series
// on small arguments, the library functions otherwise); the products are
// accumulated in double-double (two-sum) per lane, reduced across lanes in a
// fixed order, and the per-wave partial sums are added in wave order by a
// second kernel (bitwise reproducible).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "sg_internal.hpp"
#include "sg_math.hpp"

namespace sg {
namespace pts {

constexpr int KMAXP = kMaxK;
constexpr int FAM_EXP = SG_FAMILY_EXP_SUM;
constexpr int FAM_OSC = SG_FAMILY_OSCILLATORY;
constexpr int FAM_PEAK = SG_FAMILY_PRODUCT_PEAK;
constexpr int FAM_CORNER = SG_FAMILY_CORNER_PEAK;
constexpr int FAM_GAUSS = SG_FAMILY_GAUSSIAN;
constexpr int FAM_OSCQ = SG_FAMILY_OSCILLATORY_QUADRATIC;
constexpr int FAM_OSCQL = SG_FAMILY_OSCILLATORY_QUADRATIC_LINEAR;

// Families whose partial quantity is an angle (cosine of a sum).
template <int FAM>
constexpr bool is_angle() { return FAM == FAM_OSC || FAM == FAM_OSCQ || FAM == FAM_OSCQL; }
// Quadratic families: per coordinate (c, u) with the exponent c (x - u)^2
// (and, for FAM_OSCQL, a linear term l x with l[d] after u[d]).
template <int FAM>
constexpr bool is_quadratic() { return FAM == FAM_GAUSS || FAM == FAM_OSCQ || FAM == FAM_OSCQL; }
// Offset of c[0] in the parameters of a quadratic family (u follows at + d).
template <int FAM>
constexpr int quad_off() { return FAM == FAM_OSCQ || FAM == FAM_OSCQL ? 1 : 0; }

// sin(h) = h * sum_k (-h^2)^k/(2k+1)! and cos(h) = sum_k (-h^2)^k/(2k)!,
// k = 0..8, for |h| <= 0.78 (< pi/4): the first omitted terms are below
// 2^-60 of the values, and each evaluation adds about two roundings.
constexpr double kTrigSmall = 0.78;
__device__ __forceinline__ void sincos_series(double h, double& sh, double& ch)
{
    const double u = -h * h;
    double ps = inv_fact(17), pc = inv_fact(16);
#pragma unroll
    for (int k = 7; k >= 0; --k) {
        ps = fma(ps, u, inv_fact(2 * k + 1));
        pc = fma(pc, u, inv_fact(2 * k));
    }
    sh = h * ps;
    ch = pc;
}

// The same on |h| <= 1/8 with k = 0..4 for sin and k = 0..5 for cos: the
// first omitted terms, h^10/11! and h^12/12! relative, are below 2^-55.
constexpr double kTrigTiny = 0.125;
__device__ __forceinline__ void sincos_series_short(double h, double& sh, double& ch)
{
    const double u = -h * h;
    double ps = inv_fact(9), pc = inv_fact(10);
#pragma unroll
    for (int k = 3; k >= 0; --k) ps = fma(ps, u, inv_fact(2 * k + 1));
#pragma unroll
    for (int k = 4; k >= 0; --k) pc = fma(pc, u, inv_fact(2 * k));
    sh = h * ps;
    ch = pc;
}

// double-double accumulation: (hi, lo) += v exactly up to lo's rounding
__device__ __forceinline__ void dd_add(double& hi, double& lo, double v)
{
    const double t = hi + v;
    const double bp = t - hi;
    const double err = (hi - (t - bp)) + (v - bp);
    hi = t;
    lo += err;
}

// Per-wave constants of the integrand at the centre: ridge families the
// base argument (log-amplitude for exp-sum, phase for oscillatory);
// product-peak log f(c).  Lanes stride over the coordinates and the wave
// adds their sums in a fixed order (identical in every wave).
// sabs (optional) receives the sum of the magnitudes of the components,
// the scale of the value's rounding error.
template <int FAM>
__device__ __forceinline__ double centre_value(const double* __restrict__ prm, int d, double* sabs = nullptr)
{
    const int lane = threadIdx.x & 63;
    double s = 0.0, sa = 0.0;
    for (int t = lane; t < d; t += 64) {
        double v;
        if constexpr (FAM == FAM_EXP || FAM == FAM_CORNER) v = 0.5 * prm[t];
        else if constexpr (FAM == FAM_OSC) v = 0.5 * prm[1 + t];
        else if constexpr (is_quadratic<FAM>()) {
            const double hv = 0.5 - prm[quad_off<FAM>() + d + t];
            v = prm[quad_off<FAM>() + t] * (hv * hv);
            if constexpr (FAM == FAM_OSCQL) {   // the linear term's part l / 2
                const double lv = 0.5 * prm[1 + 2 * d + t];
                s += lv;
                sa += fabs(lv);
            }
        } else {
            const double b = prm[t], u = prm[d + t];
            const double hv = 0.5 - u;
            v = -log(fma(hv, hv, 1.0 / (b * b)));
        }
        s += v;
        sa += fabs(v);
    }
    for (int off = 32; off >= 1; off >>= 1) {   // same value in every lane
        s += __shfl_xor(s, off);
        sa += __shfl_xor(sa, off);
    }
    if constexpr (is_angle<FAM>()) {
        const double ph = 2.0 * 3.141592653589793 * prm[0];
        s += ph;
        sa += fabs(ph);
    }
    if (sabs) *sabs = sa;
    return s;
}

// f(x) - f(c) from the partial quantity of the point: ridge exp-sum
// e^{t0} (e^delta - 1); oscillatory cos(t0 + delta) - cos(t0) =
// -2 sin(t0 + delta/2) sin(delta/2); corner-peak (1 + t0 + delta)^-(d+1) -
// (1 + t0)^-(d+1) = f(c) (exp(-(d+1) log1p(delta / (1 + t0))) - 1);
// product-peak f(c) (e^delta - 1) with delta = sum of log(g_i(x_i) / g_i(1/2)).
//
// Oscillatory, with h = delta/2 and (s0, c0) = (sin t0, cos t0):
// sin(t0 + h) = s0 cos h + c0 sin h, so the difference is
// -2 sin h (s0 cos h + c0 sin h).  Its rounding error is at most a few
// units of |g| plus 10 u |sin h| <= 5 u |delta| (the bracket may cancel,
// but each of its two products is at most 1 in magnitude).  Exp-sum and
// product-peak: f(c) expm1(delta), at most 6 roundings of |g|.  The
// quadratic families take the same forms (gaussian as exp-sum,
// oscillatory-quadratic as oscillatory) with delta the sum of the active
// coordinates' changes c y (y + 1 - 2u) of the exponent, y = x - 1/2.
template <int FAM>
__device__ __forceinline__ double centred_value(double base, double fc, double delta, double dp1, double s0,
                                                double c0)
{
    if constexpr (is_angle<FAM>()) {
        const double h = 0.5 * delta;
        // the shorter series when every lane of the wave can take it (one
        // path per wave, no divergence)
        if (__all(fabs(h) <= kTrigTiny)) {
            double sh, ch;
            sincos_series_short(h, sh, ch);
            return -2.0 * sh * fma(s0, ch, c0 * sh);
        }
        if (fabs(h) <= kTrigSmall) {
            double sh, ch;
            sincos_series(h, sh, ch);
            return -2.0 * sh * fma(s0, ch, c0 * sh);
        }
        return -2.0 * sin(base + h) * sin(h);
    } else if constexpr (FAM == FAM_CORNER) {
        return fc * expm1(-dp1 * log1p(delta / (1.0 + base)));
    } else {
        return fc * expm1_any(delta);
    }
}

// f at the centre from the centre's argument.
template <int FAM>
__device__ __forceinline__ double centre_f(double base, int d)
{
    if constexpr (is_angle<FAM>()) return cos(base);
    else if constexpr (FAM == FAM_CORNER) return exp(-(double)(d + 1) * log1p(base));
    else return exp(base);
}

struct PointsArgs {
    int d, K, e0;
    int ri;                       // ints per unranked record: nnz, excess, K coordinates, K levels
    int off_f1, off_fc, off_sc;   // byte offsets in a wave's LDS region: 1-D frontier, group tensors, sums
    int wave_bytes;               // size of a wave's LDS region
    uint64_t n_multi, nchunks;
    const uint64_t* W;            // weak-composition counts, (K+1) rows of d+1
    const double* node_y;         // per level: x - 1/2 of its nodes
    const double* node_w;         // per level: weights
    int level_off[KMAXP + 3];     // level l occupies [level_off[l], level_off[l+1])
    double coef[KMAXP + 1];       // by excess e
    float rinv[KMAXP + 3];        // 1 / n_l (single precision) for the mixed-radix decode
    const double* params;
    double* partial;              // (hi, lo, sum of |terms|) per wave
};

// Unrank `rank` (see the canonical order above) into this lane's record:
// rec[0] = number of active coordinates, rec[1] = excess, then the K slots
// of the active coordinates (ascending) and the K slots of their levels.
__device__ __forceinline__ void unrank_into(const PointsArgs& A, uint64_t rank, int* rec)
{
    const int d = A.d, K = A.K, stride = d + 1;
    auto weak = [&](int n, int parts) -> uint64_t { return A.W[(size_t)n * stride + parts]; };
    uint64_t r = rank;
    int e = A.e0;
    for (; e < K; ++e) {
        const uint64_t c = weak(e, d);
        if (r < c) break;
        r -= c;
    }
    int i = 0, rem = e, k = 0;
    while (rem > 0 && k < K) {
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
        rec[2 + k] = j;
        rec[2 + K + k] = a + 1;
        ++k;
        rem -= a;
        i = j + 1;
    }
    rec[0] = k;
    rec[1] = e;
}

// Orders this wave's LDS writes before its later LDS reads (and the reads
// before later writes): the LDS queue of a wave is in order, so waiting for
// it to drain, with a compiler memory barrier, suffices.
__device__ __forceinline__ void wave_lds_sync()
{
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
}

template <int FAM>
__global__ void __launch_bounds__(256) k_points(PointsArgs A)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int gw = blockIdx.x * 4 + w;
    const int nw = gridDim.x * 4;
    const double* __restrict__ prm = A.params;
    const int d = A.d;

    const double base = centre_value<FAM>(prm, d);
    const double fc = centre_f<FAM>(base, d);
    const double dp1 = (double)(d + 1);
    double s0 = 0.0, c0 = 0.0;
    if constexpr (is_angle<FAM>()) {
        s0 = sin(base);
        c0 = cos(base);
    }
    unsigned char* region = smem + (size_t)w * A.wave_bytes;
    int* rec = (int*)region;
    double2* f1 = (double2*)(region + A.off_f1);    // per coordinate and node: (contribution, weight)
    double2* ft = (double2*)(region + A.off_fc);    // group tensors: (partial sum, weight product)
    double* st = (double*)(region + A.off_sc);      // group tensors: sum of |contributions|
    double hi = 0.0, lo = 0.0, aabs = 0.0;

    for (uint64_t c = gw; c < A.nchunks; c += nw) {
        const uint64_t r0 = c * 64;
        const int cnt = (int)min((uint64_t)64, A.n_multi - r0);
        wave_lds_sync();   // earlier reads of rec are done
        if (lane < cnt) unrank_into(A, r0 + lane, rec + lane * A.ri);
        wave_lds_sync();
        for (int j = 0; j < cnt; ++j) {
            const int* rj = rec + j * A.ri;
            const int nnz = __builtin_amdgcn_readfirstlane(rj[0]);
            if (nnz == 0) continue;                       // the centre: f(x) - f(c) = 0
            const int e = __builtin_amdgcn_readfirstlane(rj[1]);
            const double cw = A.coef[e];
            // active coordinates: coordinate, level, node count, offset in f1;
            // pre[m] / suf[m]: tensor sizes of coordinates [0, m) / [m, nnz)
            int nm[KMAXP], bm[KMAXP], cm[KMAXP], lm[KMAXP], pre[KMAXP + 1], suf[KMAXP + 1];
            // quadratic families: rounding scale of a coordinate's entries,
            // |c| (1 + |1 - 2u|) (the change c y (y + 1 - 2u) may cancel),
            // plus |l| for a linear term
            double es[KMAXP];
            int E = 0;
            pre[0] = 1;
#pragma unroll
            for (int m = 0; m < KMAXP; ++m) {
                es[m] = 0.0;
                if (m < nnz) {
                    cm[m] = __builtin_amdgcn_readfirstlane(rj[2 + m]);
                    lm[m] = __builtin_amdgcn_readfirstlane(rj[2 + A.K + m]);
                    nm[m] = A.level_off[lm[m] + 1] - A.level_off[lm[m]];
                    if constexpr (is_quadratic<FAM>())
                        es[m] = fabs(prm[quad_off<FAM>() + cm[m]]) *
                                (1.0 + fabs(1.0 - 2.0 * prm[quad_off<FAM>() + d + cm[m]]));
                    if constexpr (FAM == FAM_OSCQL) es[m] += fabs(prm[1 + 2 * d + cm[m]]);
                } else {
                    cm[m] = 0; lm[m] = 1; nm[m] = 1;
                }
                bm[m] = E;
                E += nm[m] * (m < nnz);
                pre[m + 1] = pre[m] * nm[m];
            }
            suf[KMAXP] = 1;
#pragma unroll
            for (int m = KMAXP - 1; m >= 0; --m) suf[m] = suf[m + 1] * nm[m];
            const int P = pre[KMAXP];
            // group A = coordinates [0, s) (the fast index), group B = [s, nnz)
            int s = 0, best = 1 + P;
#pragma unroll
            for (int m = 1; m <= KMAXP; ++m)
                if (m <= nnz && pre[m] + suf[m] < best) { best = pre[m] + suf[m]; s = m; }
            int PA = pre[0], PB = suf[0];
#pragma unroll
            for (int m = 1; m <= KMAXP; ++m)
                if (m == s) { PA = pre[m]; PB = suf[m]; }

            wave_lds_sync();   // earlier frontier reads are done
            for (int idx = lane; idx < E; idx += 64) {
                int m = 0;
#pragma unroll
                for (int mm = 1; mm < KMAXP; ++mm)
                    if (mm < nnz && idx >= bm[mm]) m = mm;
                int coord = cm[0], lev = lm[0], bb = bm[0];
#pragma unroll
                for (int mm = 1; mm < KMAXP; ++mm)
                    if (m == mm) { coord = cm[mm]; lev = lm[mm]; bb = bm[mm]; }
                const int node = A.level_off[lev] + (idx - bb);
                const double y = A.node_y[node], wt = A.node_w[node];
                double q;
                if constexpr (FAM == FAM_EXP || FAM == FAM_CORNER) q = prm[coord] * y;
                else if constexpr (FAM == FAM_OSC) q = prm[1 + coord] * y;
                else if constexpr (is_quadratic<FAM>()) {
                    // c (x - u)^2 - c (1/2 - u)^2 = c y (y + 1 - 2u)
                    const double c = prm[quad_off<FAM>() + coord], u = prm[quad_off<FAM>() + d + coord];
                    q = c * (y * (y + (1.0 - 2.0 * u)));
                    if constexpr (FAM == FAM_OSCQL) q = fma(prm[1 + 2 * d + coord], y, q);
                } else {
                    const double b = prm[coord], u = prm[d + coord];
                    const double beta = 1.0 / (b * b), hv = 0.5 - u;
                    const double yp = y + hv;
                    // g(1/2 + y) / g(1/2) - 1 = -y (2 hv + y) / (beta + (hv + y)^2)
                    q = log1p(-y * (2.0 * hv + y) / fma(yp, yp, beta));
                }
                f1[idx] = make_double2(q, wt);
            }
            wave_lds_sync();
            // the two group tensors: entries [0, PA) over group A (carrying
            // the coefficient), [PA, PA + PB) over group B
            for (int idx = lane; idx < PA + PB; idx += 64) {
                const bool inA = idx < PA;
                int rem = inA ? idx : idx - PA;
                const int m0 = inA ? 0 : s, m1 = inA ? s : nnz;
                double q = 0.0, sa = 0.0, wt = inA ? cw : 1.0;
#pragma unroll
                for (int m = 0; m < KMAXP; ++m) {
                    if (m >= m0 && m < m1) {
                        // rem = qt * n + k; rem < 2^13, so the single-precision quotient is exact
                        const int qt = (int)(((float)rem + 0.5f) * A.rinv[lm[m]]);
                        const int k = rem - qt * nm[m];
                        rem = qt;
                        const double2 f = f1[bm[m] + k];
                        q += f.x;
                        sa += fabs(f.x) + es[m];
                        wt *= f.y;
                    }
                }
                ft[idx] = make_double2(q, wt);
                st[idx] = sa;
            }
            wave_lds_sync();
            // p = ib * PA + ia; p < 2^13, so the single-precision quotient
            // (reciprocal within a few ulps) is exact after truncation
            const float rpa = 1.0f / (float)PA;
            for (int p = lane; p < P; p += 64) {
                const int ib = (int)(((float)p + 0.5f) * rpa);
                const int ia = p - ib * PA;
                const double2 a = ft[ia], b = ft[PA + ib];
                const double delta = a.x + b.x;
                const double wp = a.y * b.y;
                const double sd = st[ia] + st[PA + ib];
                const double gd = centred_value<FAM>(base, fc, delta, dp1, s0, c0);
                dd_add(hi, lo, wp * gd);
                // rounding scale of the term: its own size plus the propagated
                // error of delta (each entry and each addition rounded), times
                // |df/d delta| (oscillatory <= 1; corner-peak (d+1) f / (1 + s))
                double fx;
                if constexpr (is_angle<FAM>()) fx = 1.0;
                else if constexpr (FAM == FAM_CORNER) fx = dp1 * fabs(fc + gd) / (1.0 + base + delta);
                else fx = fabs(fc + gd);
                aabs += fabs(wp) * (fabs(gd) + fx * sd);
            }
        }
    }
    // fixed-order reduction of the lanes' double-doubles and |term| sums
    for (int off = 1; off < 64; off <<= 1) {
        const double oh = __shfl_down(hi, off), ol = __shfl_down(lo, off), oa = __shfl_down(aabs, off);
        if ((lane & (2 * off - 1)) == 0) {
            dd_add(hi, lo, oh);
            lo += ol;
            aabs += oa;
        }
    }
    if (lane == 0) {
        A.partial[3 * gw] = hi;
        A.partial[3 * gw + 1] = lo;
        A.partial[3 * gw + 2] = aabs;
    }
}

// Sum the per-wave partials in wave order (one workgroup: 256 threads each
// add a contiguous slice, then a fixed tree) and write f(c) + sum, and the
// a-priori rounding bound
//   16 u (S + |f(c)|) + e_c (|f(c)| + 1 + S),   u = 2^-53:
// a term w * g carries at most 10 roundings relative to |w g| (up to 8
// weight products, the coefficient, the product) plus g's error, at most 6
// roundings of |g| (oscillatory: 3, plus 5 u |delta|, within the next term)
// and |f(x)| times the error of the partial quantity delta (each of its at
// most 8 entries and additions, at most 6 roundings each, relative to the
// sum of the entries' magnitudes; for the quadratic families an entry's
// magnitude includes |c| (1 + |1 - 2u|), which bounds the rounding of
// c y (y + 1 - 2u) when it cancels); S accumulates
// |w| (|g| + |f(x)| sum |entry|).  e_c bounds the error of the centre's
// argument (log-amplitude or phase: a d-term sum, u (d + 4) times the sum
// of its components' magnitudes, plus 4u per logarithm); the value and every
// term move by at most |f(c)| + 1 + S per unit of it.  The double-double sum
// adds at most 2^-100 of S, the final addition one rounding.
template <int FAM>
__global__ void __launch_bounds__(256) k_points_finish(const double* __restrict__ partial, int nwaves,
                                                       const double* __restrict__ params, int d,
                                                       double* __restrict__ out, double* __restrict__ bound)
{
    __shared__ double sh[256], sl[256], sa[256];
    const int t = threadIdx.x;
    const int per = (nwaves + 255) / 256;
    double hi = 0.0, lo = 0.0, aa = 0.0;
    for (int i = t * per; i < min(nwaves, (t + 1) * per); ++i) {
        dd_add(hi, lo, partial[3 * i]);
        lo += partial[3 * i + 1];
        aa += partial[3 * i + 2];
    }
    sh[t] = hi;
    sl[t] = lo;
    sa[t] = aa;
    __syncthreads();
    for (int s = 128; s >= 1; s >>= 1) {
        if (t < s) {
            double h = sh[t], l = sl[t];
            dd_add(h, l, sh[t + s]);
            sh[t] = h;
            sl[t] = l + sl[t + s];
            sa[t] += sa[t + s];
        }
        __syncthreads();
    }
    if (t < 64) {
        double babs = 0.0;
        const double base = centre_value<FAM>(params, d, &babs);
        const double fc = centre_f<FAM>(base, d);
        if (t == 0) {
            out[0] = fc + (sh[0] + sl[0]);
            if (bound) {
                const double u = 1.1102230246251565e-16;
                const double S = sa[0] * (1.0 + 1e-12);
                double ec = u * ((double)(d + 4) * babs + (FAM == FAM_PEAK ? 4.0 * d : 0.0));
                // corner-peak: f depends on its argument through the power
                // -(d+1) (components a_i >= 0, so 1 + s >= 1), and f(c) carries
                // the rounding of (d+1) log1p(t0)
                if (FAM == FAM_CORNER) ec = (double)(d + 1) * (ec + 4.0 * u * (fabs(log1p(base)) + 1.0));
                bound[0] = 16.0 * u * (S + fabs(fc)) + ec * (fabs(fc) + 1.0 + S);
            }
        }
    }
}

}  // namespace pts


int launch_points(int family, const PointsLaunch& L, void* stream)
{
    pts::PointsArgs A;
    A.d = L.d;
    A.K = L.K;
    A.e0 = L.e0;
    auto align16 = [](int b) { return (b + 15) & ~15; };
    A.ri = 2 + 2 * L.K;
    A.off_f1 = align16(64 * A.ri * (int)sizeof(int));
    A.off_fc = A.off_f1 + 16 * std::max(1, L.emax);
    A.off_sc = A.off_fc + 16 * std::max(1, L.cmax);
    A.wave_bytes = A.off_sc + align16(8 * std::max(1, L.cmax));
    const size_t shmem = 4 * (size_t)A.wave_bytes;
    if (shmem > 65536) return (int)hipErrorInvalidValue;
    A.n_multi = L.n_multi;
    A.nchunks = (L.n_multi + 63) / 64;
    A.W = L.W;
    A.node_y = L.node_y;
    A.node_w = L.node_w;
    for (int i = 0; i < kMaxK + 3; ++i) {
        A.level_off[i] = L.level_off[i];
        const int n = i >= 1 && i <= L.K + 1 ? L.level_off[i + 1] - L.level_off[i] : 1;
        A.rinv[i] = 1.0f / (float)(n > 0 ? n : 1);
    }
    for (int i = 0; i <= kMaxK; ++i) A.coef[i] = L.coef[i];
    A.params = L.params;
    A.partial = L.partial;
    const dim3 grid((unsigned)L.grid), block(256);
    hipStream_t s = (hipStream_t)stream;
    if (family == SG_FAMILY_EXP_SUM) {
        hipLaunchKernelGGL(pts::k_points<pts::FAM_EXP>, grid, block, shmem, s, A);
        hipLaunchKernelGGL(pts::k_points_finish<pts::FAM_EXP>, dim3(1), block, 0, s, L.partial, L.grid * 4,
                           L.params, L.d, L.out, L.bound);
    } else if (family == SG_FAMILY_OSCILLATORY) {
        hipLaunchKernelGGL(pts::k_points<pts::FAM_OSC>, grid, block, shmem, s, A);
        hipLaunchKernelGGL(pts::k_points_finish<pts::FAM_OSC>, dim3(1), block, 0, s, L.partial, L.grid * 4,
                           L.params, L.d, L.out, L.bound);
    } else if (family == SG_FAMILY_PRODUCT_PEAK) {
        hipLaunchKernelGGL(pts::k_points<pts::FAM_PEAK>, grid, block, shmem, s, A);
        hipLaunchKernelGGL(pts::k_points_finish<pts::FAM_PEAK>, dim3(1), block, 0, s, L.partial, L.grid * 4,
                           L.params, L.d, L.out, L.bound);
    } else if (family == SG_FAMILY_CORNER_PEAK) {
        hipLaunchKernelGGL(pts::k_points<pts::FAM_CORNER>, grid, block, shmem, s, A);
        hipLaunchKernelGGL(pts::k_points_finish<pts::FAM_CORNER>, dim3(1), block, 0, s, L.partial, L.grid * 4,
                           L.params, L.d, L.out, L.bound);
    } else if (family == SG_FAMILY_GAUSSIAN) {
        hipLaunchKernelGGL(pts::k_points<pts::FAM_GAUSS>, grid, block, shmem, s, A);
        hipLaunchKernelGGL(pts::k_points_finish<pts::FAM_GAUSS>, dim3(1), block, 0, s, L.partial, L.grid * 4,
                           L.params, L.d, L.out, L.bound);
    } else if (family == SG_FAMILY_OSCILLATORY_QUADRATIC) {
        hipLaunchKernelGGL(pts::k_points<pts::FAM_OSCQ>, grid, block, shmem, s, A);
        hipLaunchKernelGGL(pts::k_points_finish<pts::FAM_OSCQ>, dim3(1), block, 0, s, L.partial, L.grid * 4,
                           L.params, L.d, L.out, L.bound);
    } else {
        hipLaunchKernelGGL(pts::k_points<pts::FAM_OSCQL>, grid, block, shmem, s, A);
        hipLaunchKernelGGL(pts::k_points_finish<pts::FAM_OSCQL>, dim3(1), block, 0, s, L.partial, L.grid * 4,
                           L.params, L.d, L.out, L.bound);
    }
    return (int)hipGetLastError();
}

}  // namespace sg
