// Block (tensor-product) variant of the sparse grid: the coordinates of an
// integrand are cut into consecutive blocks, each block gets its own sparse
// grid with the integrand's excess budget, and the rule is the tensor
// product of the block rules (the reading of Algorithm 3.3 with step m > 1,
// (3.8)-(3.11), under which the error grows in proportion to d/m).  For
// the product-form families the integrand factors over the blocks, so the
// value is the product of the block values, each block being an ordinary
// batched problem of the forward sweep:
//   exp-sum, product-peak, gaussian: Q = prod_b Q_b;
//   oscillatory quadratic families: Q = Re(e^{2 pi i w} prod_b
//   (R_b + i I_b)), with R_b the block's value at w = 0 and I_b the one at
//   w = -1/4 (cos(theta - pi/2) = sin theta);
//   oscillatory: the sweep's sum S_b of a block is real and the block's
//   complex value is e^{i theta_b} S_b, theta_b = sum of a_t / 2 over the
//   block (the centre phase), so one sweep per block at w = -theta_b / 2 pi
//   (phase cancelled: it returns S_b) and the combine rotates it by
//   e^{i theta_b}; Q = Re(e^{2 pi i w} prod_b e^{i theta_b} S_b).
// Two kernels surround the forward launch over the blocks: a gather that
// lays out the blocks' parameters, and a combine that forms the products in
// a fixed order and propagates the blocks' error bounds.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sg_internal.hpp"

namespace sg {
namespace blk {

// `lanes` lanes per block (a power of two, 4..64): lane j copies the block's
// coordinates j, j + lanes, ..., so each block's parameters move as
// contiguous runs (one thread per block made every lane of a wave walk its
// own strided run), and a group of lanes never straddles a wave.  The
// launcher takes the smallest power of two covering a third of the block
// size: a few independent loads per lane, and few enough waves that they
// are all resident at once.
int gather_lanes(int block_dims)
{
    int l = 4;
    while (l < 64 && 3 * l < block_dims) l *= 2;
    return l;
}

__global__ void __launch_bounds__(256) k_block_gather(const BlockSub* __restrict__ subs, int nsub, int lanes,
                                                      const double* __restrict__ params,
                                                      double* __restrict__ sub_params,
                                                      double* __restrict__ phase)
{
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t s = g / lanes;
    const int j0 = (int)(g % lanes);
    if (s >= nsub) return;
    const BlockSub b = subs[s];
    const double* src = params + b.src_off;
    double* dst = sub_params + b.dst_off;
    if (b.family == SG_FAMILY_OSCILLATORY) {
        double th = 0.0, ab = 0.0;
        for (int j = j0; j < b.len; j += lanes) {
            const double a = src[1 + b.start + j];
            dst[1 + j] = a;
            th += a;
            ab += fabs(a);
        }
        // the block's centre phase theta_b = sum a_t / 2 and sum |a_t| / 2 by
        // a fixed tree over the block's lanes (a group of `lanes` lanes
        // shares one sub-problem, so the whole group takes this branch); the
        // sweep runs at the w cancelling theta_b, the combine rotates by it
        for (int o = lanes / 2; o >= 1; o >>= 1) {
            th += __shfl_xor(th, o, lanes);
            ab += __shfl_xor(ab, o, lanes);
        }
        if (j0 == 0) {
            th *= 0.5;
            dst[0] = -th / (2.0 * 3.141592653589793);
            phase[2 * s] = th;
            phase[2 * s + 1] = 0.5 * ab;
        }
    } else if (b.family == SG_FAMILY_OSCILLATORY_QUADRATIC) {
        if (j0 == 0) dst[0] = b.part == 2 ? -0.25 : 0.0;
        for (int j = j0; j < b.len; j += lanes) {
            dst[1 + j] = src[1 + b.start + j];
            dst[1 + b.len + j] = src[1 + b.d + b.start + j];
        }
    } else if (b.family == SG_FAMILY_OSCILLATORY_QUADRATIC_LINEAR) {
        if (j0 == 0) dst[0] = b.part == 2 ? -0.25 : 0.0;
        for (int j = j0; j < b.len; j += lanes) {
            dst[1 + j] = src[1 + b.start + j];
            dst[1 + b.len + j] = src[1 + b.d + b.start + j];
            dst[1 + 2 * b.len + j] = src[1 + 2 * b.d + b.start + j];
        }
    } else if (b.family == SG_FAMILY_PRODUCT_PEAK || b.family == SG_FAMILY_GAUSSIAN) {
        for (int j = j0; j < b.len; j += lanes) {
            dst[j] = src[b.start + j];
            dst[b.len + j] = src[b.d + b.start + j];
        }
    } else {
        for (int j = j0; j < b.len; j += lanes) dst[j] = src[b.start + j];
    }
}

// Partial product of some blocks: value (complex for oscillatory), and for
// the bound P = prod |v_b| and D = prod (|v_b| + e_b) - prod |v_b|.
struct Part {
    double re, im, P, D;
};

// Joining two parts.  Real and complex products are commutative in floating
// point, so the result does not depend on which part comes first; D joins
// without cancellation: D = D1 P2 + D2 P1 + D1 D2.
__device__ __forceinline__ Part join(const Part& x, const Part& y, bool complex_value)
{
    Part r;
    if (complex_value) {
        r.re = x.re * y.re - x.im * y.im;
        r.im = x.re * y.im + x.im * y.re;
    } else {
        r.re = x.re * y.re;
        r.im = 0.0;
    }
    r.D = x.D * y.P + y.D * x.P + x.D * y.D;
    r.P = x.P * y.P;
    return r;
}

__device__ __forceinline__ Part shfl_part(const Part& x, int off)
{
    Part r;
    r.re = __shfl_down(x.re, off);
    r.im = __shfl_down(x.im, off);
    r.P = __shfl_down(x.P, off);
    r.D = __shfl_down(x.D, off);
    return r;
}

// One wave per integrand: lanes take 64 blocks at a time, a fixed lane tree
// joins them, lane 0 joins the passes in order (bitwise reproducible).
//
// Bound.  With block values v_b, |exact block value - v_b| <= e_b, the
// tensor rule's value differs from prod v_b by at most D.  Rounding of the
// k - 1 real products, in any association: at most k u (P + D); of the
// complex products (each component two products and a sum): at most
// 4 k u (P + D); of the final rotation by e^{2 pi i w}: at most
// (2 |2 pi w| + 6) u (P + D).  Every quantity of the bound is a sum or
// product of non-negative numbers, so its own rounding is covered by the
// factor 1 + 4 k u.
__global__ void __launch_bounds__(256) k_block_combine(const BlockProb* __restrict__ probs, int n,
                                                       const double* __restrict__ sub_out,
                                                       const double* __restrict__ sub_bound,
                                                       const double* __restrict__ phase,
                                                       const double* __restrict__ params,
                                                       double* __restrict__ out, double* __restrict__ bound)
{
    const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (i >= n) return;
    const BlockProb p = probs[i];
    const bool osc_lin = p.family == SG_FAMILY_OSCILLATORY;
    const bool osc = osc_lin || p.family == SG_FAMILY_OSCILLATORY_QUADRATIC ||
                     p.family == SG_FAMILY_OSCILLATORY_QUADRATIC_LINEAR;
    const double u = 1.1102230246251565e-16;
    Part acc{1.0, 0.0, 1.0, 0.0};
    for (int base = 0; base < p.nblocks; base += 64) {
        const int b = base + lane;
        Part x{1.0, 0.0, 1.0, 0.0};
        if (b < p.nblocks) {
            if (osc_lin) {
                // v_b = e^{i theta_c} q with q the phase-cancelled sweep's value
                // and theta_c the gather's sum.  Against the exact block value
                // e^{i theta} S_b: q's own bound e_b (relative to cos(delta) S_b,
                // delta = 2 pi w_b + theta the phase the cancellation leaves,
                // |delta| <= dmax; rotated by the computed sincos, |.| <= 1 + 2u),
                // sincos and the two products (<= 8 u |q|), theta_c's rounding
                // (a summation tree of len terms, <= dth = (len + 2) u A,
                // A = sum |a_t| / 2) times |S_b| <= (|q| + e_b) / cos delta, and
                // |S_b| (1 - cos delta) <= dmax^2 (|q| + e_b).
                const int s = p.first_sub + b;
                const int start = b * p.block_dims, len = min(p.block_dims, p.d - start);
                const double th = phase[2 * s], ab = phase[2 * s + 1];
                double sn, cs;
                sincos(th, &sn, &cs);
                const double q = sub_out[s], e = sub_bound[s];
                x.re = cs * q;
                x.im = sn * q;
                x.P = fabs(q) * (1.0 + 4.0 * u);
                const double dth = (double)(len + 2) * u * (ab + 1.0);
                const double dmax = 2.0 * (double)(len + 8) * u * (ab + 1.0);
                x.D = e * (1.0 + 4.0 * u) + fabs(q) * 8.0 * u + (dth + dmax * dmax) * (fabs(q) + e);
            } else if (osc) {
                const int s = p.first_sub + 2 * b;
                x.re = sub_out[s];
                x.im = sub_out[s + 1];
                x.P = hypot(x.re, x.im) * (1.0 + 2.0 * u);
                x.D = sub_bound[s] + sub_bound[s + 1];
            } else {
                const int s = p.first_sub + b;
                x.re = sub_out[s];
                x.P = fabs(x.re);
                x.D = sub_bound[s];
            }
        }
        for (int off = 1; off < 64; off <<= 1) {
            const Part y = shfl_part(x, off);
            if ((lane & (2 * off - 1)) == 0) x = join(x, y, osc);
        }
        if (lane == 0) acc = join(acc, x, osc);
    }
    if (lane != 0) return;
    const double ku = (double)p.nblocks * u;
    if (osc) {
        const double phi = 2.0 * 3.141592653589793 * params[p.param_offset];
        double sp, cp;
        sincos(phi, &sp, &cp);
        out[p.out_index] = cp * acc.re - sp * acc.im;
        if (bound) {
            const double rnd = 4.0 * ku + (2.0 * fabs(phi) + 6.0) * u;
            bound[p.out_index] = (acc.D + rnd * (acc.P + acc.D)) * (1.0 + 4.0 * ku);
        }
    } else {
        out[p.out_index] = acc.re;
        if (bound) bound[p.out_index] = (acc.D + ku * (acc.P + acc.D)) * (1.0 + 4.0 * ku);
    }
}

}  // namespace blk

int launch_block_gather(const BlockSub* subs, int nsub, int block_dims, const double* params, double* sub_params,
                        double* phase, void* stream)
{
    if (nsub <= 0) return 0;
    const int lanes = blk::gather_lanes(block_dims);
    const int64_t threads = (int64_t)nsub * lanes;
    hipLaunchKernelGGL(blk::k_block_gather, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0,
                       (hipStream_t)stream, subs, nsub, lanes, params, sub_params, phase);
    return (int)hipGetLastError();
}

int launch_block_combine(const BlockProb* probs, int n, const double* sub_out, const double* sub_bound,
                         const double* phase, const double* params, double* out, double* bound, void* stream)
{
    if (n <= 0) return 0;
    hipLaunchKernelGGL(blk::k_block_combine, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, (hipStream_t)stream, probs, n,
                       sub_out, sub_bound, phase, params, out, bound);
    return (int)hipGetLastError();
}

}  // namespace sg
