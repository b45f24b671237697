// 1-D quadrature rules of Section 2.2 on [0,1] and the difference-rule
// (hierarchical surplus) tables the dimension sweep uses.
//
// Trapezoid (2.10) and Clenshaw-Curtis (2.11) use n_1 = 1, n_l = 2^(l-1)+1
// and are nested; Gauss-Legendre (2.13) uses n_l = l in the paper, and
// n_l = 2l-1 (odd, so every level holds the centre) in the default mode.
// The paper's formulas degenerate for one point (division by n-1 = 0, or a
// single end node); level 1 is read as the midpoint with weight 1, which
// keeps the rules nested and symmetric.
#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "sg_internal.hpp"

namespace sg {

namespace {
const long double kPi = 3.141592653589793238462643383279502884L;
}

bool rule_is_known(int rule)
{
    return rule == SG_RULE_TRAPEZOID || rule == SG_RULE_CLENSHAW_CURTIS ||
           rule == SG_RULE_GAUSS_LEGENDRE || rule == SG_RULE_GAUSS_LEGENDRE_PAPER;
}

bool rule_is_nested(int rule)
{
    return rule == SG_RULE_TRAPEZOID || rule == SG_RULE_CLENSHAW_CURTIS;
}

long rule_npoints(int rule, int level)
{
    if (level < 1 || !rule_is_known(rule)) return -1;
    if (rule_is_nested(rule)) {
        if (level == 1) return 1;
        if (level > 17) return -1;
        return (1L << (level - 1)) + 1;
    }
    long n = rule == SG_RULE_GAUSS_LEGENDRE ? 2L * level - 1 : level;
    return n > 65537 ? -1 : n;
}

// Clenshaw-Curtis weights for n = N+1 points (N even) on [-1,1], written in
// the angle variable theta_j = j pi / N:
//   w_j = c_j / N * (1 - sum_{k=1}^{N/2} b_k cos(2 k theta_j) / (4k^2 - 1)),
// c_j = 1 at the two ends, 2 inside; b_k = 1 for k = N/2, 2 otherwise.
// This is (2.11) with its primed sum expanded.
static void clenshaw_curtis(long n, std::vector<long double>& x, std::vector<long double>& w)
{
    const long N = n - 1;
    x.resize(n);
    w.resize(n);
    for (long j = 0; j <= N; ++j) {
        const long double th = kPi * (long double)j / (long double)N;
        long double acc = 1.0L;
        for (long k = 1; k <= N / 2; ++k) {
            const long double b = (2 * k == N) ? 1.0L : 2.0L;
            acc -= b * std::cos(2.0L * k * th) / (4.0L * k * k - 1.0L);
        }
        const long double c = (j == 0 || j == N) ? 1.0L : 2.0L;
        // ascending nodes: x = -cos(theta) on [-1,1] -> (1 - cos theta)/2 on [0,1]
        x[j] = 0.5L - 0.5L * std::cos(th);
        w[j] = 0.5L * c * acc / (long double)N;
    }
    // exact symmetry about 1/2 (cos(pi - th) = -cos th)
    for (long j = 0; j < n / 2; ++j) {
        long double h = 0.5L * (x[n - 1 - j] - x[j]);
        x[j] = 0.5L - h;
        x[n - 1 - j] = 0.5L + h;
        long double ww = 0.5L * (w[j] + w[n - 1 - j]);
        w[j] = w[n - 1 - j] = ww;
    }
    if (n % 2 == 1) x[n / 2] = 0.5L;
}

// Gauss-Legendre: roots of P_n by Newton's method on the three-term
// recurrence, started from Tricomi's asymptotic root estimate; weights
// 2 / ((1 - t^2) P_n'(t)^2).  Only the roots t > 0 are iterated; the rule
// is completed by symmetry.
static void gauss_legendre(long n, std::vector<long double>& x, std::vector<long double>& w)
{
    x.assign(n, 0.0L);
    w.assign(n, 0.0L);
    const long m = n / 2;
    for (long i = 0; i < m; ++i) {
        // i-th largest root
        const long double k = (long double)(i + 1);
        const long double nn = (long double)n;
        long double t = (1.0L - (nn - 1.0L) / (8.0L * nn * nn * nn)) *
                        std::cos(kPi * (4.0L * k - 1.0L) / (4.0L * nn + 2.0L));
        long double dp = 1.0L;
        for (int it = 0; it < 60; ++it) {
            long double p0 = 1.0L, p1 = t;
            for (long r = 2; r <= n; ++r) {
                long double p2 = ((2.0L * r - 1.0L) * t * p1 - (r - 1.0L) * p0) / (long double)r;
                p0 = p1;
                p1 = p2;
            }
            dp = nn * (t * p1 - p0) / (t * t - 1.0L);
            long double dt = p1 / dp;
            t -= dt;
            if (std::fabs(dt) <= 1e-21L) break;
        }
        {
            long double p0 = 1.0L, p1 = t;
            for (long r = 2; r <= n; ++r) {
                long double p2 = ((2.0L * r - 1.0L) * t * p1 - (r - 1.0L) * p0) / (long double)r;
                p0 = p1;
                p1 = p2;
            }
            dp = nn * (t * p1 - p0) / (t * t - 1.0L);
        }
        const long double wt = 2.0L / ((1.0L - t * t) * dp * dp);
        // [0,1]: x = (1 + t)/2, w = wt/2; pair (1/2 - t/2, 1/2 + t/2)
        x[n - 1 - i] = 0.5L + 0.5L * t;
        x[i] = 0.5L - 0.5L * t;
        w[n - 1 - i] = w[i] = 0.5L * wt;
    }
    if (n % 2 == 1) {
        x[m] = 0.5L;
        long double s = 0.0L;
        for (long i = 0; i < n; ++i)
            if (i != m) s += w[i];
        w[m] = 1.0L - s;   // the weights sum to the interval length
    }
}

bool rule_nodes(int rule, int level, std::vector<long double>& x, std::vector<long double>& w)
{
    const long n = rule_npoints(rule, level);
    if (n < 1) return false;
    if (n == 1) {
        x.assign(1, 0.5L);
        w.assign(1, 1.0L);
        return true;
    }
    if (rule == SG_RULE_TRAPEZOID) {
        // (2.10) on [0,1]: spacing h = 1/(n-1), first and last weights halved
        const long double h = 1.0L / (long double)(n - 1);
        x.resize(n);
        w.resize(n);
        for (long j = 0; j < n; ++j) {
            x[j] = (long double)j * h;
            w[j] = (j == 0 || j == n - 1) ? 0.5L * h : h;
        }
        return true;
    }
    if (rule == SG_RULE_CLENSHAW_CURTIS) {
        clenshaw_curtis(n, x, w);
        return true;
    }
    gauss_legendre(n, x, w);
    return true;
}

// Position of a nested node as an exact integer on the finest grid of the
// table (index on the level-(K+1) grid of 2^K + 1 points).
static long nested_slot(long j, long n_level, long n_fine)
{
    return j * ((n_fine - 1) / (n_level - 1));
}

bool build_delta_table(int rule, int K, DeltaTable& t, std::string& err)
{
    if (!rule_is_known(rule)) { err = "unknown rule"; return false; }
    if (K < 0 || K > kMaxK) { err = "excess budget K out of range"; return false; }
    t = DeltaTable();
    t.rule = rule;
    t.K = K;
    t.nested = rule_is_nested(rule);
    t.level_begin.assign(K + 3, 0);

    // per level: pair list (y > 0) with the level's weight of the pair nodes
    struct PairW { long key; long double y; long double w; };
    std::vector<std::vector<PairW>> lev(K + 2);
    std::vector<long double> x, w;
    const long n_fine = rule_npoints(rule, K + 1);
    for (int l = 1; l <= K + 1; ++l) {
        if (!rule_nodes(rule, l, x, w)) { err = "rule construction failed"; return false; }
        const long n = (long)x.size();
        for (long j = 0; j < n / 2; ++j) {       // left half: x < 1/2
            PairW pw;
            pw.y = 0.5L - x[j];
            pw.w = w[j];
            pw.key = t.nested ? nested_slot(j, n, n_fine) : (long)l * 100000 + j;
            lev[l].push_back(pw);
        }
    }
    // distinct pairs in order of first appearance
    std::vector<long> keys;
    std::vector<long double> ys;
    std::vector<int> first_level;
    for (int l = 2; l <= K + 1; ++l) {
        t.level_begin[l] = (int)keys.size();
        for (const PairW& pw : lev[l]) {
            if (std::find(keys.begin(), keys.end(), pw.key) != keys.end()) continue;
            keys.push_back(pw.key);
            ys.push_back(pw.y);
            first_level.push_back(l);
        }
    }
    t.level_begin[0] = t.level_begin[1] = 0;
    t.level_begin[K + 2] = (int)keys.size();
    t.npairs = (int)keys.size();
    const int P = t.npairs;

    // weight of pair p in level l (0 if absent)
    auto wlev = [&](int l, int p) -> long double {
        if (l < 1) return 0.0L;
        for (const PairW& pw : lev[l])
            if (pw.key == keys[p]) return pw.w;
        return 0.0L;
    };
    t.y.resize(P);
    t.y32.resize(P);
    t.dw.assign((size_t)(K + 1) * P, 0.0);
    t.dw_hi.assign((size_t)(K + 1) * P, 0.0f);
    t.dw_lo.assign((size_t)(K + 1) * P, 0.0f);
    t.wabs.assign(P, 0.0);
    for (int p = 0; p < P; ++p) {
        t.y[p] = (double)ys[p];
        t.y32[p] = (float)ys[p];
        for (int e = 1; e <= K; ++e) {
            // Delta^{e+1} = J^{e+1} - J^e
            const long double v = wlev(e + 1, p) - wlev(e, p);
            const double vd = (double)v;
            t.dw[(size_t)e * P + p] = vd;
            const float hi = (float)vd;
            t.dw_hi[(size_t)e * P + p] = hi;
            t.dw_lo[(size_t)e * P + p] = (float)(vd - (double)hi);
            t.wabs[p] += std::fabs(vd);
        }
        // structural check: weights vanish outside the declared e-range
        const int L = first_level[p];
        for (int e = 1; e <= K; ++e) {
            const bool inside = t.nested ? (e >= L - 1) : (e == L - 1 || e == L);
            if (!inside && t.dw[(size_t)e * P + p] != 0.0) {
                err = "difference-rule table has weights outside its level range";
                return false;
            }
        }
    }
    return true;
}

bool build_records(const DeltaTable& t, std::vector<double>& r64, std::vector<float>& r32, std::string& err)
{
    const int rc = rule_class_of(t.rule);
    const int K = t.K, P = t.npairs;
    r64.clear();
    r32.clear();
    for (int L = 2; L <= K + 1; ++L) {
        const int b = t.level_begin[L], e = t.level_begin[L + 1];
        if (e - b != rc_pairs(rc, L) || (int)r64.size() != rc_off64(rc, K, L) ||
            (int)r32.size() != rc_off32(rc, K, L)) {
            err = "difference-rule table does not match the static layout of its rule class";
            return false;
        }
        const int lo = rc_elo(L), hi = rc_ehi(rc, K, L);
        for (int p = b; p < e; ++p) {
            r64.push_back(t.y[p]);
            for (int q = lo; q <= hi; ++q) {
                r64.push_back(t.dw[(size_t)q * P + p]);
                r32.push_back(t.dw_hi[(size_t)q * P + p]);
                r32.push_back(t.dw_lo[(size_t)q * P + p]);
            }
            r64.push_back(t.wabs[p]);
        }
    }
    return true;
}

}  // namespace sg
