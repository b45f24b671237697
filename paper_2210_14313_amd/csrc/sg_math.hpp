// Small device math shared by the kernels: Taylor series and a
// branch-free expm1 with a stated rounding budget.
#pragma once

#include <hip/hip_runtime.h>

namespace sg {

// 1/k!, exact factorials (k <= 20) rounded once
constexpr double inv_fact(int k)
{
    double f = 1.0;
    for (int i = 2; i <= k; ++i) f *= (double)i;
    return 1.0 / f;
}

// expm1(x) for |x| <= 1/2: x * sum_{k=1..16} x^(k-1)/k!; the first omitted
// term is below 2^-64 of the sum, Horner's rule adds about one rounding and
// the final product one more.
constexpr double kExpSmall = 0.5;
__device__ __forceinline__ double expm1_series(double x)
{
    double p = inv_fact(16);
#pragma unroll
    for (int k = 15; k >= 1; --k) p = fma(p, x, inv_fact(k));
    return x * p;
}

// expm1(x) for any x: x itself on |x| <= 1/2; otherwise x = k ln2 + r with
// k = rint(x / ln2) != 0 and |r| <= 0.35 (ln2 split in two parts, the first
// with 12 trailing zero bits so that k times it is exact), and
// expm1(x) = 2^k expm1(r) + (2^k - 1).  The two terms have the same sign
// except for k = 1, r < 0 and k = -1, r > 0 (x within [0.5, 1.04] in
// magnitude), where the sum is at least 0.39 and at most 2.1 times smaller
// than the terms' magnitudes: at most 5 roundings of the result in all cases.
// No branch: every lane runs the same instructions.
constexpr double kLn2Hi = 0x1.62e42fefa3000p-1;
constexpr double kLn2Lo = 0x1.3de6af278ece6p-42;
constexpr double kLog2e = 1.4426950408889634;
__device__ __forceinline__ double expm1_any(double x)
{
    const double kd = fabs(x) <= kExpSmall ? 0.0 : rint(x * kLog2e);
    const double r = fma(-kd, kLn2Lo, fma(-kd, kLn2Hi, x));
    const double e = expm1_series(r);
    const int k = (int)kd;
    const double t = ldexp(e, k) + (ldexp(1.0, k) - 1.0);
    return kd == 0.0 ? e : t;
}

}  // namespace sg
