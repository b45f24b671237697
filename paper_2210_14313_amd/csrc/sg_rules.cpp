// 1-D quadrature rules of Section 2.2 on [0,1] and the difference-rule
// (hierarchical surplus) tables the dimension sweep uses.
//
// Trapezoid (2.10) and Clenshaw-Curtis (2.11) use n_1 = 1, n_l = 2^(l-1)+1
// and are nested; Gauss-Legendre (2.13) uses n_l = l in the paper, and
// n_l = 2l-1 (odd, so every level holds the centre) in the default mode;
// Gauss-Patterson (2.12) is nested, with the level-to-points map listed in
// Section 5.4 (1, 3, 3, 7, 7, 7, 15, 15, 15, 15 for levels 1..10).
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
    return rule == SG_RULE_TRAPEZOID || rule == SG_RULE_CLENSHAW_CURTIS || rule == SG_RULE_GAUSS_PATTERSON ||
           rule == SG_RULE_GAUSS_LEGENDRE || rule == SG_RULE_GAUSS_LEGENDRE_PAPER;
}

bool rule_is_nested(int rule)
{
    return rule == SG_RULE_TRAPEZOID || rule == SG_RULE_CLENSHAW_CURTIS || rule == SG_RULE_GAUSS_PATTERSON;
}

long rule_npoints(int rule, int level)
{
    if (level < 1 || !rule_is_known(rule)) return -1;
    if (rule == SG_RULE_GAUSS_PATTERSON) {
        static const long kMap[11] = {0, 1, 3, 3, 7, 7, 7, 15, 15, 15, 15};
        return level <= 10 ? kMap[level] : -1;
    }
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

// Gauss-Patterson rules of 1, 3, 7 and 15 points (Example 3 of Section
// 2.2), on [0,1].  Each step adds to the symmetric n-point rule (n odd,
// nodes t_i on [-1,1]) the n+1 zeros of the polynomial G of degree n+1 that
// is orthogonal to all lower degrees with respect to the weight
// pi(t) = prod (t - t_i).  pi is odd and G even, so with G written in the
// Chebyshev basis, G = T_{n+1} + sum_{j even} c_j T_j, the conditions are
//   int_{-1}^{1} pi(t) G(t) T_k(t) dt = 0,   k odd <= n,
// (n+1)/2 linear equations whose integrals a Gauss-Legendre rule evaluates
// exactly.  The zeros of G interlace with the old nodes (one between 0 and
// the first positive node, one between consecutive ones, one above the
// last) and are found by bisection.  Weights: the integrals of the Lagrange
// basis polynomials, by a Gauss-Legendre rule exact for their degree.
static void chebyshev_all(int m, long double t, long double* T)
{
    T[0] = 1.0L;
    if (m >= 1) T[1] = t;
    for (int k = 2; k <= m; ++k) T[k] = 2.0L * t * T[k - 1] - T[k - 2];
}

static bool gauss_patterson(long N, std::vector<long double>& x, std::vector<long double>& w)
{
    std::vector<long double> gx, gw;
    gauss_legendre(32, gx, gw);              // on [0,1]; exact for degree 63 >= 3n + 1
    std::vector<long double> t(1, 0.0L);     // nodes on [-1,1]
    long n = 1;
    long double T[64];
    while (n < N) {
        const int m = (int)n + 1, h = m / 2;
        std::vector<long double> A((size_t)h * h, 0.0L), rhs(h, 0.0L);
        for (size_t g = 0; g < gx.size(); ++g) {
            const long double u = 2.0L * gx[g] - 1.0L, wg = 2.0L * gw[g];
            long double pi = 1.0L;
            for (long double ti : t) pi *= u - ti;
            chebyshev_all(m, u, T);
            for (int r = 0; r < h; ++r) {
                const long double f = wg * pi * T[2 * r + 1];
                for (int c = 0; c < h; ++c) A[(size_t)r * h + c] += f * T[2 * c];
                rhs[r] -= f * T[m];
            }
        }
        for (int c = 0; c < h; ++c) {        // elimination with partial pivoting
            int piv = c;
            for (int r = c + 1; r < h; ++r)
                if (std::fabs(A[(size_t)r * h + c]) > std::fabs(A[(size_t)piv * h + c])) piv = r;
            if (A[(size_t)piv * h + c] == 0.0L) return false;
            for (int j = 0; j < h; ++j) std::swap(A[(size_t)c * h + j], A[(size_t)piv * h + j]);
            std::swap(rhs[c], rhs[piv]);
            for (int r = c + 1; r < h; ++r) {
                const long double f = A[(size_t)r * h + c] / A[(size_t)c * h + c];
                for (int j = c; j < h; ++j) A[(size_t)r * h + j] -= f * A[(size_t)c * h + j];
                rhs[r] -= f * rhs[c];
            }
        }
        std::vector<long double> c(h, 0.0L);
        for (int r = h - 1; r >= 0; --r) {
            long double sum = rhs[r];
            for (int j = r + 1; j < h; ++j) sum -= A[(size_t)r * h + j] * c[j];
            c[r] = sum / A[(size_t)r * h + r];
        }
        auto G = [&](long double u) {
            chebyshev_all(m, u, T);
            long double v = T[m];
            for (int j = 0; j < h; ++j) v += c[j] * T[2 * j];
            return v;
        };
        std::vector<long double> ends(1, 0.0L);
        for (long double ti : t)
            if (ti > 0.0L) ends.push_back(ti);
        std::sort(ends.begin(), ends.end());
        ends.push_back(1.0L);
        std::vector<long double> added;
        for (size_t iv = 0; iv + 1 < ends.size(); ++iv) {
            long double lo = ends[iv], hi = ends[iv + 1];
            long double glo = G(lo), ghi = G(hi);
            if (glo == 0.0L || ghi == 0.0L || (glo > 0.0L) == (ghi > 0.0L)) return false;
            for (int it = 0; it < 128; ++it) {
                const long double mid = 0.5L * (lo + hi), gm = G(mid);
                if ((gm > 0.0L) == (glo > 0.0L)) { lo = mid; glo = gm; } else hi = mid;
            }
            added.push_back(0.5L * (lo + hi));
        }
        for (long double v : added) {
            t.push_back(v);
            t.push_back(-v);
        }
        n = (long)t.size();
    }
    if (n != N) return false;
    std::sort(t.begin(), t.end());
    x.assign(N, 0.5L);
    for (long i = 0; i < N; ++i) x[i] = i == N / 2 ? 0.5L : 0.5L + 0.5L * t[i];
    // Lagrange integrals on [0,1] by a Gauss-Legendre rule exact for degree N - 1
    std::vector<long double> lx, lw;
    gauss_legendre(N + 1, lx, lw);
    w.assign(N, 0.0L);
    for (long i = 0; i < N; ++i) {
        long double sum = 0.0L;
        for (size_t k = 0; k < lx.size(); ++k) {
            long double L = 1.0L;
            for (long j = 0; j < N; ++j)
                if (j != i) L *= (lx[k] - x[j]) / (x[i] - x[j]);
            sum += lw[k] * L;
        }
        w[i] = sum;
    }
    return true;
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
    if (rule == SG_RULE_GAUSS_PATTERSON) return gauss_patterson(n, x, w);
    gauss_legendre(n, x, w);
    return true;
}

// Position of a nested node as an exact integer on the finest grid of the
// table (index on the level-(K+1) grid).  Trapezoid and Clenshaw-Curtis:
// node j of n sits at j (n_fine - 1)/(n - 1).  Gauss-Patterson: each
// extension interlaces its new nodes with the old ones, so node j of n sits
// at (j + 1)(n_fine + 1)/(n + 1) - 1.
static long nested_slot(int rule, long j, long n_level, long n_fine)
{
    if (rule == SG_RULE_GAUSS_PATTERSON) return (j + 1) * ((n_fine + 1) / (n_level + 1)) - 1;
    if (n_level == 1) return (n_fine - 1) / 2;
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
            pw.key = t.nested ? nested_slot(rule, j, n, n_fine) : (long)l * 100000 + j;
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
