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
// ridge integrand, or log(g_i(x)/g_i(1/2)) of a product integrand), so a
// point costs one LDS read per active coordinate.  Lanes cover the tensor
// points; f(x) - f(c) is formed without cancellation from the partial
// quantity; the products are accumulated in double-double (two-sum) per lane,
// reduced across lanes in a fixed order, and the per-wave partial sums are
// added in wave order by a second kernel (bitwise reproducible).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sg_internal.hpp"

namespace sg {
namespace pts {

constexpr int KMAXP = kMaxK;
constexpr int FAM_EXP = SG_FAMILY_EXP_SUM;
constexpr int FAM_OSC = SG_FAMILY_OSCILLATORY;
constexpr int FAM_PEAK = SG_FAMILY_PRODUCT_PEAK;
constexpr int FAM_CORNER = SG_FAMILY_CORNER_PEAK;

constexpr int REC_INTS = 2 + 2 * KMAXP;   // per unranked multi-index: nnz, excess, coords, levels

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
        else {
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
    if constexpr (FAM == FAM_OSC) {
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
template <int FAM>
__device__ __forceinline__ double centred_value(double base, double fc, double delta, double dp1)
{
    if constexpr (FAM == FAM_OSC) return -2.0 * sin(base + 0.5 * delta) * sin(0.5 * delta);
    else if constexpr (FAM == FAM_CORNER) return fc * expm1(-dp1 * log1p(delta / (1.0 + base)));
    else return fc * expm1(delta);
}

// f at the centre from the centre's argument.
template <int FAM>
__device__ __forceinline__ double centre_f(double base, int d)
{
    if constexpr (FAM == FAM_OSC) return cos(base);
    else if constexpr (FAM == FAM_CORNER) return exp(-(double)(d + 1) * log1p(base));
    else return exp(base);
}

struct PointsArgs {
    int d, K, e0;
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
// rec[0] = number of active coordinates, rec[1] = excess, then the active
// coordinates (ascending) and their levels.
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
    while (rem > 0 && k < KMAXP) {
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
        rec[2 + KMAXP + k] = a + 1;
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

constexpr int FRONTIER_MAX = 264;   // >= max over multi-indices of the sum of n_l (K <= 8: 257)

template <int FAM>
__global__ void __launch_bounds__(256) k_points(PointsArgs A)
{
    __shared__ int recs[4][64 * REC_INTS];
    __shared__ double2 front[4][FRONTIER_MAX];
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int gw = blockIdx.x * 4 + w;
    const int nw = gridDim.x * 4;
    const double* __restrict__ prm = A.params;
    const int d = A.d;

    const double base = centre_value<FAM>(prm, d);
    const double fc = centre_f<FAM>(base, d);
    const double dp1 = (double)(d + 1);
    int* rec = recs[w];
    double2* fr = front[w];
    double hi = 0.0, lo = 0.0, aabs = 0.0;

    for (uint64_t c = gw; c < A.nchunks; c += nw) {
        const uint64_t r0 = c * 64;
        const int cnt = (int)min((uint64_t)64, A.n_multi - r0);
        wave_lds_sync();   // earlier reads of rec are done
        if (lane < cnt) unrank_into(A, r0 + lane, rec + lane * REC_INTS);
        wave_lds_sync();
        for (int j = 0; j < cnt; ++j) {
            const int* rj = rec + j * REC_INTS;
            const int nnz = __builtin_amdgcn_readfirstlane(rj[0]);
            if (nnz == 0) continue;                       // the centre: f(x) - f(c) = 0
            const int e = __builtin_amdgcn_readfirstlane(rj[1]);
            const double cw = A.coef[e];
            // stage the frontier: nodes of every active coordinate
            int nm[KMAXP], bm[KMAXP], cm[KMAXP], lm[KMAXP];
            int E = 0, P = 1;
#pragma unroll
            for (int m = 0; m < KMAXP; ++m) {
                if (m < nnz) {
                    cm[m] = __builtin_amdgcn_readfirstlane(rj[2 + m]);
                    lm[m] = __builtin_amdgcn_readfirstlane(rj[2 + KMAXP + m]);
                    nm[m] = A.level_off[lm[m] + 1] - A.level_off[lm[m]];
                    bm[m] = E;
                    E += nm[m];
                    P *= nm[m];
                } else {
                    cm[m] = 0; lm[m] = 1; nm[m] = 1; bm[m] = E;
                }
            }
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
                else {
                    const double b = prm[coord], u = prm[d + coord];
                    const double beta = 1.0 / (b * b), hv = 0.5 - u;
                    const double yp = y + hv;
                    // g(1/2 + y) / g(1/2) - 1 = -y (2 hv + y) / (beta + (hv + y)^2)
                    q = log1p(-y * (2.0 * hv + y) / fma(yp, yp, beta));
                }
                fr[idx] = make_double2(q, wt);
            }
            wave_lds_sync();
            for (int p = lane; p < P; p += 64) {
                int rem = p;
                double delta = 0.0, sd = 0.0, wp = cw;
#pragma unroll
                for (int m = 0; m < KMAXP; ++m) {
                    if (m < nnz) {
                        // rem = qt * n + k; P < 2^13, so the single-precision quotient is exact
                        const int qt = (int)(((float)rem + 0.5f) * A.rinv[lm[m]]);
                        const int k = rem - qt * nm[m];
                        rem = qt;
                        const double2 f = fr[bm[m] + k];
                        delta += f.x;
                        sd += fabs(f.x);
                        wp *= f.y;
                    }
                }
                const double gd = centred_value<FAM>(base, fc, delta, dp1);
                dd_add(hi, lo, wp * gd);
                // rounding scale of the term: its own size plus the propagated
                // error of delta (each entry and each addition rounded), times
                // |df/d delta| (oscillatory <= 1; corner-peak (d+1) f / (1 + s))
                double fx;
                if constexpr (FAM == FAM_OSC) fx = 1.0;
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
// weight products, the coefficient, the product) plus g's error, at most 4
// roundings of |g| and |f(x)| times the error of the partial quantity delta
// (each of its at most 8 entries and additions, at most 6 roundings each,
// relative to the sum of the entries' magnitudes); S accumulates
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
        hipLaunchKernelGGL(pts::k_points<pts::FAM_EXP>, grid, block, 0, s, A);
        hipLaunchKernelGGL(pts::k_points_finish<pts::FAM_EXP>, dim3(1), block, 0, s, L.partial, L.grid * 4,
                           L.params, L.d, L.out, L.bound);
    } else if (family == SG_FAMILY_OSCILLATORY) {
        hipLaunchKernelGGL(pts::k_points<pts::FAM_OSC>, grid, block, 0, s, A);
        hipLaunchKernelGGL(pts::k_points_finish<pts::FAM_OSC>, dim3(1), block, 0, s, L.partial, L.grid * 4,
                           L.params, L.d, L.out, L.bound);
    } else if (family == SG_FAMILY_PRODUCT_PEAK) {
        hipLaunchKernelGGL(pts::k_points<pts::FAM_PEAK>, grid, block, 0, s, A);
        hipLaunchKernelGGL(pts::k_points_finish<pts::FAM_PEAK>, dim3(1), block, 0, s, L.partial, L.grid * 4,
                           L.params, L.d, L.out, L.bound);
    } else {
        hipLaunchKernelGGL(pts::k_points<pts::FAM_CORNER>, grid, block, 0, s, A);
        hipLaunchKernelGGL(pts::k_points_finish<pts::FAM_CORNER>, dim3(1), block, 0, s, L.partial, L.grid * 4,
                           L.params, L.d, L.out, L.bound);
    }
    return (int)hipGetLastError();
}

}  // namespace sg
