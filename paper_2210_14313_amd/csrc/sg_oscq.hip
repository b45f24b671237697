// Oscillatory-quadratic sweep (with or without the linear term): the FP64
// forward launchers, the dispatch over precision modes, and the complex
// reverse sweep (FP64 in every mode).
#include "sg_oscq_dev.hpp"

namespace sg {

// the FP32 modes' kernels are compiled in their own units
extern template int launch_oscq_prec<SG_PREC_FP32_COMPENSATED>(int, int, int, int, int, const double*, const float*,
                                                               const double*, double*, double*, double*, void*);
extern template int launch_oscq_prec<SG_PREC_FP32_FP64_SUM>(int, int, int, int, int, const double*, const float*,
                                                            const double*, double*, double*, double*, void*);
extern template int launch_oscq_batch_prec<SG_PREC_FP32_COMPENSATED>(int, const OscqDesc*, const double*,
                                                                     const float*, const double*, double*, double*,
                                                                     void*);
extern template int launch_oscq_batch_prec<SG_PREC_FP32_FP64_SUM>(int, const OscqDesc*, const double*, const float*,
                                                                  const double*, double*, double*, void*);

template int launch_oscq_prec<SG_PREC_FP64>(int, int, int, int, int, const double*, const float*, const double*,
                                            double*, double*, double*, void*);
template int launch_oscq_batch_prec<SG_PREC_FP64>(int, const OscqDesc*, const double*, const float*, const double*,
                                                  double*, double*, void*);

int launch_oscq(int precision, int d, int K, int rule, int G, int lin, const double* pool64, const float* pool32,
                const double* params, double* out, double* bound, double* scratch, void* stream)
{
    switch (precision) {
    case SG_PREC_FP64:
        return launch_oscq_prec<SG_PREC_FP64>(d, K, rule, G, lin, pool64, pool32, params, out, bound, scratch, stream);
    case SG_PREC_FP32_COMPENSATED:
        return launch_oscq_prec<SG_PREC_FP32_COMPENSATED>(d, K, rule, G, lin, pool64, pool32, params, out, bound,
                                                          scratch, stream);
    case SG_PREC_FP32_FP64_SUM:
        return launch_oscq_prec<SG_PREC_FP32_FP64_SUM>(d, K, rule, G, lin, pool64, pool32, params, out, bound,
                                                       scratch, stream);
    default:
        return (int)hipErrorInvalidValue;
    }
}

int launch_oscq_batch(int precision, int n, const OscqDesc* descs, const double* pool64, const float* pool32,
                      const double* params, double* out, double* bound, void* stream)
{
    switch (precision) {
    case SG_PREC_FP64:
        return launch_oscq_batch_prec<SG_PREC_FP64>(n, descs, pool64, pool32, params, out, bound, stream);
    case SG_PREC_FP32_COMPENSATED:
        return launch_oscq_batch_prec<SG_PREC_FP32_COMPENSATED>(n, descs, pool64, pool32, params, out, bound, stream);
    case SG_PREC_FP32_FP64_SUM:
        return launch_oscq_batch_prec<SG_PREC_FP32_FP64_SUM>(n, descs, pool64, pool32, params, out, bound, stream);
    default:
        return (int)hipErrorInvalidValue;
    }
}

namespace dev {

// ------------------------------------------------------------ reverse sweep
// Gradient of Q = Re(E S), E = e^{i Phi}, Phi = 2 pi w + sum_t (a_t hv_t^2 + c_t / 2)
// (hv = 1/2 - u), S = sum_{b <= K} [z^b] prod_t D_t(z):
//   dQ/dw = -2 pi Im(E S);
//   dQ/dp_t = Re(E (i dPhi/dp_t S + sum_e G_t[e] d delta_t[e]/dp_t)),
// with G_t[e] = sum_{j <= K-e} [z^j] R_t and R_t = prod_{t' != t} D_t' from
// exclusive prefix and suffix products (no division), dPhi/da_t = hv_t^2,
// dPhi/du_t = -2 a_t hv_t, dPhi/dc_t = 1/2, and per pair (t1 = a y^2,
// t2 = beta y, beta = a b + c, b = 2 hv)
//   d pair/da = 2 e^{i t1} (i y^2 cos t2 - b y sin t2),
//   d pair/dc = -2 y e^{i t1} sin t2,
//   d pair/du = -2 a d pair/dc (t2 depends on u through beta only), so the
// surpluses' u-derivatives are -2 a times their c-derivatives.

// Derivative surpluses of one coordinate with respect to a and c.
template <int K, int RC>
__device__ __forceinline__ void dsurplus_oscq(const double* __restrict__ r64, double a, double b, double beta,
                                              double (&ar)[MAXK + 1], double (&ai)[MAXK + 1],
                                              double (&cr)[MAXK + 1], double (&ci)[MAXK + 1])
{
#pragma unroll
    for (int e = 0; e <= MAXK; ++e) { ar[e] = 0.0; ai[e] = 0.0; cr[e] = 0.0; ci[e] = 0.0; }
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
            sincos(beta * y, &s2, &c2);
            const double pr = -b * y * s2, pi = y * y * c2;     // i y^2 cos t2 - b y sin t2
            const double dar = 2.0 * (c1 * pr - s1 * pi), dai = 2.0 * (c1 * pi + s1 * pr);
            const double f = -2.0 * y * s2;
            const double dcr = f * c1, dci = f * s1;
#pragma unroll
            for (int e = lo; e <= hi; ++e) {
                const double w = r[1 + e - lo];
                ar[e] = fma(w, dar, ar[e]);
                ai[e] = fma(w, dai, ai[e]);
                cr[e] = fma(w, dcr, cr[e]);
                ci[e] = fma(w, dci, ci[e]);
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
    const bool lin = q.lin != 0;
    for (int t = tid; t < d; t += 256) {
        const double a = prm[1 + t], hv = 0.5 - prm[1 + d + t];
        const double c = lin ? prm[1 + 2 * d + t] : 0.0;
        const double ab = a * (2.0 * hv);
        double dr[MAXK + 1], di[MAXK + 1], e_t = 0.0;
        int opaque = 0;
        asm volatile("" : "+s"(opaque));
        surplus_oscq<K, RC>(r64 + opaque, a, ab + c, fabs(ab) + fabs(c), dr, di, e_t);
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
        ph += fma(0.5, c, a * (hv * hv));
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
        const double c = lin ? prm[1 + 2 * d + t] : 0.0;
        double ar[MAXK + 1], ai[MAXK + 1], cr[MAXK + 1], ci[MAXK + 1];
        int opaque = 0;
        asm volatile("" : "+s"(opaque));
        dsurplus_oscq<K, RC>(r64 + opaque, a, 2.0 * hv, fma(a, 2.0 * hv, c), ar, ai, cr, ci);
        double da_r = 0.0, da_i = 0.0, dc_r = 0.0, dc_i = 0.0;
#pragma unroll
        for (int e = 1; e <= K; ++e) {
            da_r = fma(Gr[e], ar[e], fma(-Gi[e], ai[e], da_r));
            da_i = fma(Gr[e], ai[e], fma(Gi[e], ar[e], da_i));
            dc_r = fma(Gr[e], cr[e], fma(-Gi[e], ci[e], dc_r));
            dc_i = fma(Gr[e], ci[e], fma(Gi[e], cr[e], dc_i));
        }
        // Z = i dPhi S + dS; dQ = Re(E Z) = cos Phi Re Z - sin Phi Im Z
        const double pa = hv * hv, pu = -2.0 * a * hv, mu = -2.0 * a;
        const double za_r = da_r - pa * s_im, za_i = da_i + pa * s_re;
        const double zu_r = fma(mu, dc_r, -pu * s_im), zu_i = fma(mu, dc_i, pu * s_re);
        grad[q.param_offset + 1 + t] = g * fma(cs, za_r, -sn * za_i);
        grad[q.param_offset + 1 + d + t] = g * fma(cs, zu_r, -sn * zu_i);
        if (lin) {
            const double zc_r = fma(-0.5, s_im, dc_r), zc_i = fma(0.5, s_re, dc_i);
            grad[q.param_offset + 1 + 2 * d + t] = g * fma(cs, zc_r, -sn * zc_i);
        }
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

int launch_oscq_grad(int n, const OscqDesc* descs, const double* pool64, const double* params, const double* gout,
                     double* grad, double* ws, void* stream)
{
    if (n <= 0) return 0;
    hipLaunchKernelGGL(dev::k_oscq_grad, dim3((unsigned)n), dim3(256), 0, (hipStream_t)stream, descs, pool64, params,
                       gout, grad, ws);
    return (int)hipGetLastError();
}

}  // namespace sg
