/*
 * CPU oracle for Smolyak sparse-grid quadrature -- TEST INFRASTRUCTURE ONLY.
 *
 * Nothing in the product library calls this file.  Only the test suite, the
 * smoke check and the benchmark's CPU baseline load it (through ctypes).  It
 * shares no code, header, table or constant with the GPU library.
 *
 * What it computes is the plain definition of the Smolyak rule of
 * Section 2.1, equations (2.6)-(2.7):
 *
 *   Q_d^q(f) = sum_{q-d+1 <= |l| <= q} (-1)^(q-|l|) C(d-1, q-|l|)
 *              sum_{|l| fixed} (J^{l_1} x ... x J^{l_d}) f,
 *
 * with each tensor sub-rule (2.7) summed point by point.  Two evaluations
 * are offered:
 *
 *   or_smolyak_points      the definition, point by point, in x87 extended
 *                          precision (64-bit mantissa), OpenMP-free pthreads;
 *   or_smolyak_factorised  the same definition for product / exponential-ridge
 *                          integrands, where each tensor sub-rule of a product
 *                          of 1-D factors is the product of 1-D rule values
 *                          (a finite Fubini step), and the sum over all
 *                          multi-indices of one level sum is a coefficient of
 *                          a polynomial product; done in IEEE binary128.
 *
 * 1-D rules (Section 2.2) are rebuilt here from their formulas, on [0,1]:
 *   trapezoidal (2.10), Clenshaw-Curtis (2.11), Gauss-Legendre (2.13) with
 *   n_l = l (the paper's count) or n_l = 2l-1.  Level 1 of every rule is the
 *   midpoint with weight 1 (the paper's formulas degenerate at n = 1).
 *
 * Integrand families (unit cube):
 *   exp-sum       f(x) = exp(sum c_i x_i)
 *   oscillatory   f(x) = cos(2 pi w + sum a_i x_i)
 *   product-peak  f(x) = prod 1/(b_i^-2 + (x_i - u_i)^2)     ((4.4), (5.2))
 *   monomial      f(x) = prod (x_i - s)^alpha_i   (point path only, never
 *                 centred; params alpha[d], s) -- for polynomial exactness
 *   corner-peak   f(x) = (1 + sum a_i x_i)^-(d+1)            (params a[d])
 *   gaussian      f(x) = exp(sum c_i (x_i - u_i)^2)           ((4.1)-(4.3);
 *                 params c[d], u[d], c of either sign)
 *   oscillatory-quadratic  f(x) = cos(2 pi w + sum a_i (x_i - u_i)^2)
 *                 ((4.1), (4.2); params w, a[d], u[d])
 *   oscillatory-quadratic-linear
 *                 f(x) = cos(2 pi w + sum a_i (x_i - u_i)^2 + sum c_i x_i)
 *                 (the sine of (4.2) with its linear term; params w, a[d],
 *                 u[d], c[d])
 *
 * Build: gcc -O2 -fPIC -shared -ffp-contract=off sg_oracle.c -lquadmath -lpthread -lm
 */
#include <math.h>
#include <pthread.h>
#include <quadmath.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef __float128 f128;
typedef long double fld;

enum { OR_TR = 1, OR_CC = 2, OR_GP = 3, OR_GL = 4, OR_GL_PAPER = 5 };
enum { OR_EXP = 0, OR_OSC = 1, OR_PEAK = 2, OR_MONO = 3, OR_CORNER = 4, OR_GAUSS = 5, OR_OSCQ = 6, OR_OSCQL = 7 };

#define OR_MAX_LEVEL 16
#define OR_MAX_NODES 40000

/* ------------------------------------------------------------------ */
/* 1-D rules                                                           */
/* ------------------------------------------------------------------ */

/* Number of points of the level-l rule (Section 2.2). */
long or_rule_npoints(int rule, int level)
{
    if (level < 1) return -1;
    switch (rule) {
    case OR_TR:
    case OR_CC:
        if (level == 1) return 1;
        if (level > 24) return -1;
        return (1L << (level - 1)) + 1;         /* (2.10), (2.11): 2^(l-1)+1 */
    case OR_GL: return 2L * level - 1;           /* 2l-1 points */
    case OR_GL_PAPER: return level;              /* (2.13): n_l = l */
    case OR_GP: {
        /* (2.12) with the level-to-points map of Section 5.4:
         * q = 1..10 <-> N = 1, 3, 3, 7, 7, 7, 15, 15, 15, 15 */
        static const long map[11] = {0, 1, 3, 3, 7, 7, 7, 15, 15, 15, 15};
        return level <= 10 ? map[level] : -1;
    }
    default: return -1;
    }
}

/* Legendre polynomial P_n and its derivative at t, three-term recurrence. */
static void legendre_q(int n, f128 t, f128 *p, f128 *dp)
{
    f128 p0 = 1, p1 = t;
    if (n == 0) { *p = 1; *dp = 0; return; }
    for (int k = 2; k <= n; ++k) {
        f128 p2 = ((2 * k - 1) * t * p1 - (k - 1) * p0) / k;
        p0 = p1; p1 = p2;
    }
    *p = p1;
    *dp = n * (t * p1 - p0) / (t * t - 1);
}

/* Legendre polynomials P_0..P_m at t (three-term recurrence). */
static void legendre_all_q(int m, f128 t, f128 *P)
{
    P[0] = 1;
    if (m >= 1) P[1] = t;
    for (int k = 2; k <= m; ++k) P[k] = ((2 * k - 1) * t * P[k - 1] - (k - 1) * P[k - 2]) / k;
}

/* Gaussian elimination with partial pivoting on an n x n system (row-major
 * A, right-hand side b, solution in b).  Returns 0, or -1 if singular. */
static int solve_q(int n, f128 *A, f128 *b)
{
    for (int c = 0; c < n; ++c) {
        int piv = c;
        for (int r = c + 1; r < n; ++r)
            if (fabsq(A[r * n + c]) > fabsq(A[piv * n + c])) piv = r;
        if (A[piv * n + c] == 0) return -1;
        if (piv != c) {
            for (int j = 0; j < n; ++j) { f128 t = A[c * n + j]; A[c * n + j] = A[piv * n + j]; A[piv * n + j] = t; }
            f128 t = b[c]; b[c] = b[piv]; b[piv] = t;
        }
        for (int r = c + 1; r < n; ++r) {
            f128 f = A[r * n + c] / A[c * n + c];
            for (int j = c; j < n; ++j) A[r * n + j] -= f * A[c * n + j];
            b[r] -= f * b[c];
        }
    }
    for (int r = n - 1; r >= 0; --r) {
        f128 s = b[r];
        for (int j = r + 1; j < n; ++j) s -= A[r * n + j] * b[j];
        b[r] = s / A[r * n + r];
    }
    return 0;
}

/*
 * One Kronrod-Patterson extension on [-1,1] (Example 3 of Section 2.2): the
 * n (odd) symmetric nodes t[] of the previous rule, with node polynomial
 * pi(t) = prod (t - t_i), gain the n+1 zeros of the polynomial G of degree
 * n+1 orthogonal to every polynomial of degree <= n with respect to the
 * weight pi.  G is written in the Legendre basis, G = P_{n+1} + sum c_j P_j;
 * pi is odd and G even, so only even j and the conditions against odd P_k
 * remain: (n+1)/2 linear equations, their integrals taken by a Gauss-Legendre
 * rule exact for the degree.  The new zeros interlace with the old nodes (one
 * between consecutive positive old nodes, one beyond the last, one below the
 * first) and are found by bisection.  Returns the new node count, or -1.
 */
/* G(u) = P_m(u) + sum_c b[c] P_{2c}(u). */
static f128 g_at(int m, int h, const f128 *b, f128 u)
{
    f128 P[64];
    legendre_all_q(m, u, P);
    f128 s = P[m];
    for (int c = 0; c < h; ++c) s += b[c] * P[2 * c];
    return s;
}

static int patterson_extend_q(int n, const f128 *t, f128 *tn)
{
    enum { NG = 48 };
    static __thread f128 gx[NG], gw[NG];
    static __thread int gl_ready = 0;
    if (!gl_ready) {
        f128 xq[NG], wq[NG];
        for (long i = 1; i <= NG; ++i) {
            f128 u = cosq(M_PIq * (i - 0.25Q) / (NG + 0.5Q));
            for (int it = 0; it < 100; ++it) {
                f128 p, dp;
                legendre_q(NG, u, &p, &dp);
                f128 du = p / dp;
                u -= du;
                if (fabsq(du) < 1e-33Q) break;
            }
            f128 p, dp;
            legendre_q(NG, u, &p, &dp);
            xq[i - 1] = u;
            wq[i - 1] = 2 / ((1 - u * u) * dp * dp);
        }
        for (int i = 0; i < NG; ++i) { gx[i] = xq[i]; gw[i] = wq[i]; }
        gl_ready = 1;
    }
    const int m = n + 1, h = (n + 1) / 2;
    if (3 * n + 1 > 2 * NG - 1 || h > 32) return -1;
    f128 A[32 * 32], b[32], P[64];
    for (int r = 0; r < h; ++r) {
        const int k = 2 * r + 1;                    /* odd P_k */
        for (int c = 0; c < h; ++c) A[r * h + c] = 0;
        b[r] = 0;
        for (int g = 0; g < NG; ++g) {
            f128 pi = 1;
            for (int i = 0; i < n; ++i) pi *= gx[g] - t[i];
            legendre_all_q(m, gx[g], P);
            const f128 f = gw[g] * pi * P[k];
            for (int c = 0; c < h; ++c) A[r * h + c] += f * P[2 * c];   /* even P_j, j = 2c < m */
            b[r] -= f * P[m];
        }
    }
    if (solve_q(h, A, b) != 0) return -1;
    /* positive old nodes, ascending */
    f128 pos[32];
    int np = 0;
    for (int i = 0; i < n; ++i) if (t[i] > 0) pos[np++] = t[i];
    for (int i = 1; i < np; ++i) for (int j = i; j > 0 && pos[j] < pos[j - 1]; --j) {
        f128 tt = pos[j]; pos[j] = pos[j - 1]; pos[j - 1] = tt;
    }
    if (np + 1 != h) return -1;
    int cnt = 0;
    for (int iv = 0; iv <= np; ++iv) {
        f128 lo = iv == 0 ? 0 : pos[iv - 1], hi = iv == np ? 1 : pos[iv];
        f128 glo, ghi;
        glo = g_at(m, h, b, lo);
        ghi = g_at(m, h, b, hi);
        if (glo == 0 || ghi == 0 || (glo > 0) == (ghi > 0)) return -1;   /* no sign change: not interlacing */
        for (int it = 0; it < 240; ++it) {
            f128 mid = (lo + hi) / 2, gm;
            gm = g_at(m, h, b, mid);
            if ((gm > 0) == (glo > 0)) { lo = mid; glo = gm; } else hi = mid;
        }
        tn[cnt++] = (lo + hi) / 2;
        tn[cnt++] = -(lo + hi) / 2;
    }
    return cnt;
}

/* Gauss-Patterson rule of N = 1, 3, 7 or 15 points on [0,1]: the midpoint,
 * then Patterson extensions; interpolatory weights from the Legendre moment
 * equations sum_i w_i P_k(t_i) = 2 [k = 0], k < N (well conditioned). */
static int patterson_q(long N, f128 *x, f128 *w)
{
    f128 t[32], tn[32];
    int n = 1;
    t[0] = 0;
    while (n < N) {
        int k = patterson_extend_q(n, t, tn);
        if (k != n + 1) return -1;
        for (int i = 0; i < k; ++i) t[n + i] = tn[i];
        n += k;
    }
    if (n != N) return -1;
    for (int i = 1; i < n; ++i) for (int j = i; j > 0 && t[j] < t[j - 1]; --j) {
        f128 tt = t[j]; t[j] = t[j - 1]; t[j - 1] = tt;
    }
    f128 A[32 * 32], b[32], P[32];
    for (int i = 0; i < n; ++i) {
        legendre_all_q(n - 1, t[i], P);
        for (int k = 0; k < n; ++k) A[k * n + i] = P[k];
    }
    for (int k = 0; k < n; ++k) b[k] = k == 0 ? 2 : 0;
    if (solve_q(n, A, b) != 0) return -1;
    for (int i = 0; i < n; ++i) {
        x[i] = (1 + t[i]) / 2;
        w[i] = b[i] / 2;
    }
    x[n / 2] = 0.5Q;
    return n;
}

/*
 * Level-l nodes and weights on [0,1] in binary128.  Returns n, or -1.
 * Nodes are sorted ascending.
 */
int or_rule_q(int rule, int level, f128 *x, f128 *w)
{
    long n = or_rule_npoints(rule, level);
    if (n < 1 || n > OR_MAX_NODES) return -1;
    if (n == 1) { x[0] = 0.5Q; w[0] = 1; return 1; }
    const f128 pi = M_PIq;
    if (rule == OR_TR) {
        /* (2.10): equal spacing h, end weights halved; on [0,1] h = 1/(n-1) */
        f128 h = 1.0Q / (n - 1);
        for (long j = 0; j < n; ++j) {
            x[j] = j * h;
            w[j] = (j == 0 || j == n - 1) ? h / 2 : h;
        }
        return (int)n;
    }
    if (rule == OR_CC) {
        /* (2.11) on [-1,1]: x_j = -cos(pi (j-1)/(n-1)),
         * w_1 = w_n = 1/(n(n-2)),
         * w_j = 2/(n-1) (1 + 2 sum'_{k=1}^{(n-1)/2} cos(2 pi (j-1) k/(n-1))/(1-4k^2)),
         * the last term of the primed sum halved.  Mapped to [0,1]: x -> (1+x)/2,
         * w -> w/2. */
        long m = (n - 1) / 2;
        for (long j = 1; j <= n; ++j) {
            f128 xs = -cosq(pi * (j - 1) / (n - 1));
            f128 ws;
            if (j == 1 || j == n) {
                ws = 1.0Q / ((f128)n * (n - 2));
            } else {
                f128 s = 0;
                for (long k = 1; k <= m; ++k) {
                    f128 term = cosq(2 * pi * (j - 1) * k / (n - 1)) / (1 - 4.0Q * k * k);
                    if (k == m) term /= 2;
                    s += term;
                }
                ws = 2.0Q / (n - 1) * (1 + 2 * s);
            }
            x[j - 1] = (1 + xs) / 2;
            w[j - 1] = ws / 2;
        }
        return (int)n;
    }
    if (rule == OR_GP) return patterson_q(n, x, w);
    if (rule == OR_GL || rule == OR_GL_PAPER) {
        /* (2.13): zeros of P_n, Newton iteration from Chebyshev-like guesses;
         * weights 2/((1-t^2) P_n'(t)^2) on [-1,1]. */
        for (long i = 1; i <= n; ++i) {
            f128 t = cosq(pi * (i - 0.25Q) / (n + 0.5Q));
            for (int it = 0; it < 100; ++it) {
                f128 p, dp;
                legendre_q((int)n, t, &p, &dp);
                f128 dt = p / dp;
                t -= dt;
                if (fabsq(dt) < 1e-33Q) break;
            }
            f128 p, dp;
            legendre_q((int)n, t, &p, &dp);
            f128 wt = 2 / ((1 - t * t) * dp * dp);
            /* i-th root in descending order -> ascending index n-i */
            x[n - i] = (1 + t) / 2;
            w[n - i] = wt / 2;
        }
        if (n % 2 == 1) x[n / 2] = 0.5Q;   /* the centre root is exactly 0 */
        return (int)n;
    }
    return -1;
}

/* Double-precision copy of a rule, for tests. */
int or_rule(int rule, int level, double *x, double *w)
{
    static __thread f128 xq[OR_MAX_NODES], wq[OR_MAX_NODES];
    int n = or_rule_q(rule, level, xq, wq);
    for (int j = 0; j < n; ++j) { x[j] = (double)xq[j]; w[j] = (double)wq[j]; }
    return n;
}

/* ------------------------------------------------------------------ */
/* Multi-index enumeration, canonical order                            */
/* ------------------------------------------------------------------ */
/*
 * The window of (2.6) is q-d+1 <= |l| <= q, i.e. excess e = |l|-d in
 * [max(0, K-d+1), K] with K = q-d.  Canonical order: by excess ascending;
 * within one excess, by (l_1, ..., l_d) lexicographically DEcreasing.
 * A multi-index is reported sparsely: the coordinates with l_i >= 2
 * (ascending) and their levels.
 *
 * Enumeration walks, for the current remaining excess `rem`, the next
 * coordinate j >= i that is raised above level 1 and its extra level
 * k = rem..1; this visits compositions in exactly the decreasing-lex order.
 */
typedef void (*or_visit_fn)(void *ctx, int e, int nnz, const int *coords, const int *levels);

typedef struct {
    int d;
    int coords[64], levels[64];
    or_visit_fn fn;
    void *ctx;
    int e;
} enum_state;

static void enum_rec(enum_state *s, int i, int rem, int depth)
{
    if (rem == 0) { s->fn(s->ctx, s->e, depth, s->coords, s->levels); return; }
    for (int j = i; j < s->d; ++j) {
        for (int k = rem; k >= 1; --k) {
            s->coords[depth] = j;
            s->levels[depth] = k + 1;
            enum_rec(s, j + 1, rem - k, depth + 1);
        }
    }
}

static void enumerate_window(int d, int q, or_visit_fn fn, void *ctx)
{
    int K = q - d;
    int e0 = K - d + 1 > 0 ? K - d + 1 : 0;
    enum_state s;
    s.d = d; s.fn = fn; s.ctx = ctx;
    for (int e = e0; e <= K; ++e) { s.e = e; enum_rec(&s, 0, e, 0); }
}

typedef struct {
    uint64_t rank, start, count;
    int max_nnz;
    int32_t *coords, *levels, *nnz;
} enum_out;

static void enum_collect(void *ctx, int e, int nnz, const int *coords, const int *levels)
{
    (void)e;
    enum_out *o = (enum_out *)ctx;
    if (o->rank >= o->start && o->rank < o->start + o->count) {
        uint64_t r = o->rank - o->start;
        o->nnz[r] = nnz;
        for (int k = 0; k < nnz && k < o->max_nnz; ++k) {
            o->coords[r * o->max_nnz + k] = coords[k];
            o->levels[r * o->max_nnz + k] = levels[k];
        }
    }
    o->rank++;
}

/*
 * Enumerate the window in canonical order and return the multi-indices with
 * rank in [start, start+count) (sparse, padded to max_nnz per row).
 * Returns the total number of multi-indices in the window.  Only for small
 * cases: the whole window is walked.  K must be < 64.
 */
uint64_t or_enumerate(int d, int q, uint64_t start, uint64_t count, int max_nnz,
                      int32_t *coords, int32_t *levels, int32_t *nnz)
{
    if (d < 1 || q < d || q - d >= 64) return 0;
    enum_out o = {0, start, count, max_nnz, coords, levels, nnz};
    enumerate_window(d, q, enum_collect, &o);
    return o.rank;
}

/* ------------------------------------------------------------------ */
/* Exact binomials                                                     */
/* ------------------------------------------------------------------ */
static unsigned __int128 binom_u128(long n, long k)
{
    if (k < 0 || k > n) return 0;
    if (k > n - k) k = n - k;
    unsigned __int128 r = 1;
    for (long i = 1; i <= k; ++i) r = r * (unsigned __int128)(n - k + i) / (unsigned __int128)i;
    return r;
}

/* Signed combination coefficient of (2.6) for excess e, as a long double. */
static fld comb_coef(int d, int K, int e)
{
    unsigned __int128 c = binom_u128(d - 1, K - e);
    fld v = (fld)c;
    return ((K - e) % 2) ? -v : v;
}

/* ------------------------------------------------------------------ */
/* Point-by-point evaluation of (2.6)-(2.7)                            */
/* ------------------------------------------------------------------ */
typedef struct {
    int d, q, K, rule, family, centred;
    const double *params;
    /* rules per level, extended precision */
    int n[OR_MAX_LEVEL + 1];
    fld *x[OR_MAX_LEVEL + 1], *w[OR_MAX_LEVEL + 1];
    fld fc;          /* f at the centre (1/2,...,1/2) */
    fld theta_c;     /* oscillatory: 2 pi w + sum a_i / 2 */
} pt_problem;

typedef struct {
    const pt_problem *P;
    int tid, nthreads;
    uint64_t ordinal;
    fld sum, comp;        /* Neumaier sum of coef * T_l */
    fld absum;            /* sum of |coef| sum |prod w| |value| */
    uint64_t npoints;
} pt_worker;

static inline void neumaier(fld *s, fld *c, fld v)
{
    fld t = *s + v;
    if (fabsl(*s) >= fabsl(v)) *c += (*s - t) + v; else *c += (v - t) + *s;
    *s = t;
}

/* Value used for one point; `xs` are the active coordinates' positions. */
static fld point_value(const pt_problem *P, int m, const int *coords, const fld *xs)
{
    const double *p = P->params;
    int d = P->d;
    if (P->family == OR_EXP) {
        if (!P->centred) {
            fld t = 0;
            for (int i = 0; i < d; ++i) t += (fld)p[i] * 0.5L;
            for (int k = 0; k < m; ++k) t += (fld)p[coords[k]] * (xs[k] - 0.5L);
            return expl(t);
        }
        fld t = 0;
        for (int k = 0; k < m; ++k) t += (fld)p[coords[k]] * (xs[k] - 0.5L);
        return P->fc * expm1l(t);                     /* f(x) - f(c) */
    }
    if (P->family == OR_OSC) {
        fld t = 0;
        for (int k = 0; k < m; ++k) t += (fld)p[1 + coords[k]] * (xs[k] - 0.5L);
        if (!P->centred) return cosl(P->theta_c + t);
        /* cos(A + t) - cos(A) = -2 sin(t/2) sin(A + t/2) */
        return -2.0L * sinl(0.5L * t) * sinl(P->theta_c + 0.5L * t);
    }
    if (P->family == OR_GAUSS || P->family == OR_OSCQ || P->family == OR_OSCQL) {
        /* the exponent's change from the centre: with y = x - 1/2,
         * c (x - u)^2 - c (1/2 - u)^2 = c y (y + 1 - 2u), plus l y for a
         * linear term l x */
        const double *cc = P->family == OR_GAUSS ? p : p + 1;
        const double *uu = cc + d;
        fld t = 0;
        for (int k = 0; k < m; ++k) {
            int i = coords[k];
            fld y = xs[k] - 0.5L;
            t += (fld)cc[i] * y * (y + 1.0L - 2.0L * (fld)uu[i]);
            if (P->family == OR_OSCQL) t += (fld)cc[2 * d + i] * y;
        }
        if (P->family == OR_GAUSS) {
            if (!P->centred) return expl(P->theta_c + t);
            return P->fc * expm1l(t);
        }
        if (!P->centred) return cosl(P->theta_c + t);
        return -2.0L * sinl(0.5L * t) * sinl(P->theta_c + 0.5L * t);
    }
    if (P->family == OR_CORNER) {
        /* f(x) = (1 + sum a_i x_i)^-(d+1), a ridge function of s = t_c + t */
        fld t = 0;
        for (int k = 0; k < m; ++k) t += (fld)p[coords[k]] * (xs[k] - 0.5L);
        if (!P->centred) return powl(1.0L + P->theta_c + t, -(fld)(d + 1));
        /* f(x) - f(c) = f(c) ((1 + t / (1 + t_c))^-(d+1) - 1) */
        return P->fc * expm1l(-(fld)(d + 1) * log1pl(t / (1.0L + P->theta_c)));
    }
    if (P->family == OR_MONO) {
        /* every coordinate: inactive ones sit at the level-1 node 1/2 */
        const double s = p[d];
        fld v = 1;
        int k = 0;
        for (int i = 0; i < d; ++i) {
            fld xi = 0.5L;
            if (k < m && coords[k] == i) xi = xs[k++];
            int a = (int)p[i];
            for (int r = 0; r < a; ++r) v *= (xi - (fld)s);
        }
        return v;
    }
    /* product peak */
    {
        const double *b = p, *u = p + d;
        if (!P->centred) {
            fld v = P->fc;
            for (int k = 0; k < m; ++k) {
                int i = coords[k];
                fld bi = (fld)b[i], ui = (fld)u[i];
                fld Dc = 1.0L / (bi * bi) + (0.5L - ui) * (0.5L - ui);
                fld Dx = 1.0L / (bi * bi) + (xs[k] - ui) * (xs[k] - ui);
                v *= Dc / Dx;
            }
            return v;
        }
        /* f(x)/f(c) - 1 = prod (1 + h_i) - 1 with
         * h_i = (1/2 - x)(1/2 + x - 2u) / D_i(x); accumulate r <- r + h + r h */
        fld r = 0;
        for (int k = 0; k < m; ++k) {
            int i = coords[k];
            fld bi = (fld)b[i], ui = (fld)u[i];
            fld Dx = 1.0L / (bi * bi) + (xs[k] - ui) * (xs[k] - ui);
            fld h = (0.5L - xs[k]) * (0.5L + xs[k] - 2.0L * ui) / Dx;
            r = r + h + r * h;
        }
        return P->fc * r;
    }
}

static void pt_visit(void *ctx, int e, int m, const int *coords, const int *levels)
{
    pt_worker *W = (pt_worker *)ctx;
    uint64_t ord = W->ordinal++;
    if ((ord / 64) % (uint64_t)W->nthreads != (uint64_t)W->tid) return;
    const pt_problem *P = W->P;
    fld coef = comb_coef(P->d, P->K, e);

    /* tensor sub-rule (2.7) over the active coordinates; the others sit at
     * the level-1 node 1/2 with weight 1 */
    int idx[64];
    fld xs[64];
    for (int k = 0; k < m; ++k) idx[k] = 0;
    fld T = 0, Tc = 0, Tabs = 0;
    uint64_t npts = 0;
    for (;;) {
        fld wp = 1;
        for (int k = 0; k < m; ++k) {
            xs[k] = P->x[levels[k]][idx[k]];
            wp *= P->w[levels[k]][idx[k]];
        }
        fld v = point_value(P, m, coords, xs);
        neumaier(&T, &Tc, wp * v);
        Tabs += fabsl(wp * v);
        ++npts;
        int k = 0;
        for (; k < m; ++k) {
            if (++idx[k] < P->n[levels[k]]) break;
            idx[k] = 0;
        }
        if (k == m) break;
    }
    neumaier(&W->sum, &W->comp, coef * (T + Tc));
    W->absum += fabsl(coef) * Tabs;
    W->npoints += npts;
}

static void *pt_thread(void *arg)
{
    pt_worker *W = (pt_worker *)arg;
    enumerate_window(W->P->d, W->P->q, pt_visit, W);
    return NULL;
}

/*
 * Point-by-point Smolyak sum (2.6)-(2.7).
 *   rule: 1 trapezoidal, 2 Clenshaw-Curtis, 4 Gauss-Legendre (2l-1), 5 Gauss-Legendre (l)
 *   family: 0 exp-sum (params c[d]), 1 oscillatory (w, a[d]), 2 product-peak (b[d], u[d]),
 *           4 corner-peak (a[d] >= 0: f = (1 + sum a_i x_i)^-(d+1))
 *   centred: 1 -> sum f(x) - f(c) and add f(c) once (uses that the weights of
 *            the whole rule sum to 1); 0 -> sum f(x) itself.
 * out[0], out[1]: Q as a double-double (hi, lo)
 * out[2]: A = sum_l |coef_l| sum_j |prod w| |value|  (rounding-error scale)
 * out[3]: f(c);  out[4]: number of points visited (with repetition)
 * Returns 0, or -1 on bad arguments.
 */
int or_smolyak_points(int d, int q, int rule, int family, const double *params,
                      int nthreads, int centred, double *out)
{
    if (d < 1 || q < d || !params || !out) return -1;
    int K = q - d;
    if (K + 1 > OR_MAX_LEVEL || K >= 64) return -1;
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    pt_problem P;
    memset(&P, 0, sizeof(P));
    P.d = d; P.q = q; P.K = K; P.rule = rule; P.family = family; P.centred = centred;
    P.params = params;
    f128 *xq = malloc(sizeof(f128) * OR_MAX_NODES), *wq = malloc(sizeof(f128) * OR_MAX_NODES);
    int ok = 1;
    for (int l = 1; l <= K + 1; ++l) {
        int n = or_rule_q(rule, l, xq, wq);
        if (n < 1) { ok = 0; break; }
        P.n[l] = n;
        P.x[l] = malloc(sizeof(fld) * n);
        P.w[l] = malloc(sizeof(fld) * n);
        for (int j = 0; j < n; ++j) { P.x[l][j] = (fld)xq[j]; P.w[l][j] = (fld)wq[j]; }
    }
    free(xq); free(wq);
    if (!ok) return -1;
    if (family == OR_EXP) {
        fld t = 0;
        for (int i = 0; i < d; ++i) t += (fld)params[i] * 0.5L;
        P.fc = expl(t);
    } else if (family == OR_OSC) {
        fld t = 2.0L * 3.14159265358979323846264338327950288L * (fld)params[0];
        for (int i = 0; i < d; ++i) t += (fld)params[1 + i] * 0.5L;
        P.theta_c = t;
        P.fc = cosl(t);
    } else if (family == OR_PEAK) {
        fld v = 1;
        for (int i = 0; i < d; ++i) {
            fld bi = (fld)params[i], ui = (fld)params[d + i];
            v /= 1.0L / (bi * bi) + (0.5L - ui) * (0.5L - ui);
        }
        P.fc = v;
    } else if (family == OR_CORNER) {
        fld t = 0;
        for (int i = 0; i < d; ++i) t += (fld)params[i] * 0.5L;
        P.theta_c = t;
        P.fc = powl(1.0L + t, -(fld)(d + 1));
    } else if (family == OR_GAUSS || family == OR_OSCQ || family == OR_OSCQL) {
        const double *cc = family == OR_GAUSS ? params : params + 1;
        fld t = family != OR_GAUSS ? 2.0L * 3.14159265358979323846264338327950288L * (fld)params[0] : 0.0L;
        for (int i = 0; i < d; ++i) {
            fld h = 0.5L - (fld)cc[d + i];
            t += (fld)cc[i] * h * h;
            if (family == OR_OSCQL) t += (fld)cc[2 * d + i] * 0.5L;
        }
        P.theta_c = t;
        P.fc = family == OR_GAUSS ? expl(t) : cosl(t);
    } else if (family == OR_MONO) {
        P.centred = centred = 0;
        P.fc = 0;
    } else {
        return -1;
    }

    pt_worker *W = calloc(nthreads, sizeof(pt_worker));
    pthread_t *th = calloc(nthreads, sizeof(pthread_t));
    for (int t = 0; t < nthreads; ++t) {
        W[t].P = &P; W[t].tid = t; W[t].nthreads = nthreads;
        pthread_create(&th[t], NULL, pt_thread, &W[t]);
    }
    fld s = 0, c = 0, A = 0;
    uint64_t np = 0;
    for (int t = 0; t < nthreads; ++t) {
        pthread_join(th[t], NULL);
    }
    for (int t = 0; t < nthreads; ++t) {       /* fixed order: deterministic */
        neumaier(&s, &c, W[t].sum);
        neumaier(&s, &c, W[t].comp);
        A += W[t].absum;
        np += W[t].npoints;
    }
    if (centred) neumaier(&s, &c, P.fc);
    fld Q = s + c;
    double hi = (double)Q;
    out[0] = hi;
    out[1] = (double)(Q - (fld)hi);
    out[2] = (double)A;
    out[3] = (double)P.fc;
    out[4] = (double)np;
    free(W); free(th);
    for (int l = 1; l <= K + 1; ++l) { free(P.x[l]); free(P.w[l]); }
    return 0;
}

/* ------------------------------------------------------------------ */
/* Factorised evaluation in binary128                                  */
/* ------------------------------------------------------------------ */
/*
 * For f = prod_t g_t(x_t) the tensor rule (2.7) factorises:
 *   (J^{l_1} x ... x J^{l_d}) f = prod_t J^{l_t}(g_t),
 * and summing over all l with |l| - d = e gives the z^e coefficient of
 *   P(z) = prod_t U_t(z),  U_t(z) = sum_{k>=0} J^{k+1}(g_t) z^k.
 * Hence Q = sum_{e in window} (-1)^(K-e) C(d-1, K-e) [z^e] P(z).
 * The exponential-sum family is such a product with g_t(x) = exp(c_t x);
 * the oscillatory one is the real part of exp(2 pi i w) prod exp(i a_t x).
 * Complex numbers are carried as (re, im) pairs.
 */
typedef struct { f128 re, im; } cq;
static inline cq cq_mul(cq a, cq b) { cq r = {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; return r; }
static inline cq cq_add(cq a, cq b) { cq r = {a.re + b.re, a.im + b.im}; return r; }

typedef struct {
    int d, K, rule, family;
    const double *params;
    int n[OR_MAX_LEVEL + 1];
    f128 *x[OR_MAX_LEVEL + 1], *w[OR_MAX_LEVEL + 1];
} fq_problem;

static int fq_setup(fq_problem *F, int d, int q, int rule, int family, const double *params)
{
    memset(F, 0, sizeof(*F));
    if (d < 1 || q < d || q - d + 1 > OR_MAX_LEVEL) return -1;
    if (!(family == OR_EXP || family == OR_OSC || family == OR_PEAK || family == OR_GAUSS || family == OR_OSCQ ||
          family == OR_OSCQL))
        return -1;
    F->d = d; F->K = q - d; F->rule = rule; F->family = family; F->params = params;
    for (int l = 1; l <= F->K + 1; ++l) {
        long n = or_rule_npoints(rule, l);
        if (n < 1 || n > OR_MAX_NODES) return -1;
        F->x[l] = malloc(sizeof(f128) * n);
        F->w[l] = malloc(sizeof(f128) * n);
        F->n[l] = or_rule_q(rule, l, F->x[l], F->w[l]);
    }
    return 0;
}

static void fq_free(fq_problem *F)
{
    for (int l = 1; l <= F->K + 1; ++l) { free(F->x[l]); free(F->w[l]); }
}

/* g_t(x) and its derivatives with respect to the coordinate's parameters.
 * exp: g = e^{c x}, dg/dc = x g.  osc: g = e^{i a x}, dg/da = i x g.
 * peak: g = 1/(b^-2 + (x-u)^2), dg/db = 2 b^-3 g^2, dg/du = 2 (x-u) g^2.
 * gaussian: g = e^{c (x-u)^2}, dg/dc = (x-u)^2 g, dg/du = -2 c (x-u) g.
 * oscillatory-quadratic: g = e^{i a (x-u)^2}, dg/da = i (x-u)^2 g,
 * dg/du = -2 i a (x-u) g; with a linear term, g = e^{i (a (x-u)^2 + c x)},
 * the same two and dg/dc = i x g. */
static void fq_factor(const fq_problem *F, int t, f128 x, cq *g, cq *dg1, cq *dg2, cq *dg3)
{
    const double *p = F->params;
    cq z = {0, 0};
    *dg1 = z; *dg2 = z; *dg3 = z;
    if (F->family == OR_EXP) {
        f128 c = p[t];
        f128 v = expq(c * x);
        g->re = v; g->im = 0;
        dg1->re = x * v;
    } else if (F->family == OR_OSC) {
        f128 a = p[1 + t];
        g->re = cosq(a * x); g->im = sinq(a * x);
        dg1->re = -x * g->im; dg1->im = x * g->re;
    } else if (F->family == OR_GAUSS) {
        f128 c = p[t], u = p[F->d + t], v = x - u;
        f128 e = expq(c * v * v);
        g->re = e; g->im = 0;
        dg1->re = v * v * e;
        dg2->re = -2 * c * v * e;
    } else if (F->family == OR_OSCQ || F->family == OR_OSCQL) {
        f128 a = p[1 + t], u = p[1 + F->d + t], v = x - u;
        f128 ph = a * v * v;
        if (F->family == OR_OSCQL) ph += (f128)p[1 + 2 * F->d + t] * x;
        g->re = cosq(ph); g->im = sinq(ph);
        dg1->re = -v * v * g->im; dg1->im = v * v * g->re;
        dg2->re = 2 * a * v * g->im; dg2->im = -2 * a * v * g->re;
        dg3->re = -x * g->im; dg3->im = x * g->re;
    } else {
        f128 b = p[t], u = p[F->d + t];
        f128 D = 1 / (b * b) + (x - u) * (x - u);
        f128 v = 1 / D;
        g->re = v; g->im = 0;
        dg1->re = 2 / (b * b * b) * v * v;
        dg2->re = 2 * (x - u) * v * v;
    }
}

/* U_t coefficients k = 0..K (and their parameter derivatives). */
static void fq_U(const fq_problem *F, int t, cq *U, cq *dU1, cq *dU2, cq *dU3)
{
    for (int k = 0; k <= F->K; ++k) {
        cq s = {0, 0}, s1 = {0, 0}, s2 = {0, 0}, s3 = {0, 0};
        int l = k + 1;
        for (int j = 0; j < F->n[l]; ++j) {
            cq g, g1, g2, g3;
            fq_factor(F, t, F->x[l][j], &g, &g1, &g2, &g3);
            f128 wj = F->w[l][j];
            s.re += wj * g.re; s.im += wj * g.im;
            s1.re += wj * g1.re; s1.im += wj * g1.im;
            s2.re += wj * g2.re; s2.im += wj * g2.im;
            s3.re += wj * g3.re; s3.im += wj * g3.im;
        }
        U[k] = s;
        if (dU1) dU1[k] = s1;
        if (dU2) dU2[k] = s2;
        if (dU3) dU3[k] = s3;
    }
}

static void poly_mul_trunc(cq *acc, const cq *b, int K)
{
    cq r[64];
    for (int i = 0; i <= K; ++i) { r[i].re = 0; r[i].im = 0; }
    for (int i = 0; i <= K; ++i)
        for (int j = 0; i + j <= K; ++j) r[i + j] = cq_add(r[i + j], cq_mul(acc[i], b[j]));
    for (int i = 0; i <= K; ++i) acc[i] = r[i];
}

/* sum_{e in window} coef_e P[e], as a complex binary128 number */
static cq fq_combine(const fq_problem *F, const cq *P)
{
    int d = F->d, K = F->K;
    int e0 = K - d + 1 > 0 ? K - d + 1 : 0;
    cq s = {0, 0};
    for (int e = e0; e <= K; ++e) {
        unsigned __int128 c = binom_u128(d - 1, K - e);
        f128 cf = (f128)c;
        if ((K - e) % 2) cf = -cf;
        s.re += cf * P[e].re; s.im += cf * P[e].im;
    }
    return s;
}

/*
 * Factorised value.  out[0], out[1]: Q as (hi, lo) doubles.
 * Returns 0, or -1 on bad arguments.
 */
int or_smolyak_factorised(int d, int q, int rule, int family, const double *params, double *out)
{
    fq_problem F;
    if (fq_setup(&F, d, q, rule, family, params)) { fq_free(&F); return -1; }
    int K = F.K;
    cq P[64], U[64];
    for (int k = 0; k <= K; ++k) { P[k].re = 0; P[k].im = 0; }
    P[0].re = 1;
    for (int t = 0; t < d; ++t) {
        fq_U(&F, t, U, NULL, NULL, NULL);
        poly_mul_trunc(P, U, K);
    }
    cq s = fq_combine(&F, P);
    f128 Q;
    if (family == OR_OSC || family == OR_OSCQ || family == OR_OSCQL) {
        f128 ph = 2 * M_PIq * (f128)params[0];
        Q = cosq(ph) * s.re - sinq(ph) * s.im;
    } else {
        Q = s.re;
    }
    out[0] = (double)Q;
    out[1] = (double)(Q - (f128)out[0]);
    fq_free(&F);
    return 0;
}

/*
 * Factorised gradient of Q with respect to every parameter, same layout as
 * params (exp: dc[d]; osc: dw, da[d]; peak: db[d], du[d]; gaussian: dc[d],
 * du[d]; oscillatory-quadratic: dw, da[d], du[d], and with the linear term
 * dc[d] after them).  Differentiates
 * the factorised sum: dP/dp_t = dU_t(z) * prod_{s != t} U_s(z), with the
 * products excluding t formed from prefix and suffix products.
 */
int or_smolyak_factorised_grad(int d, int q, int rule, int family, const double *params, double *grad)
{
    fq_problem F;
    if (fq_setup(&F, d, q, rule, family, params)) { fq_free(&F); return -1; }
    int K = F.K, L = K + 1;
    cq *U = malloc(sizeof(cq) * (size_t)d * L), *dU1 = malloc(sizeof(cq) * (size_t)d * L),
       *dU2 = malloc(sizeof(cq) * (size_t)d * L), *dU3 = malloc(sizeof(cq) * (size_t)d * L);
    cq *pre = malloc(sizeof(cq) * (size_t)(d + 1) * L), *suf = malloc(sizeof(cq) * (size_t)(d + 1) * L);
    for (int t = 0; t < d; ++t)
        fq_U(&F, t, U + (size_t)t * L, dU1 + (size_t)t * L, dU2 + (size_t)t * L, dU3 + (size_t)t * L);
    for (int k = 0; k < L; ++k) {
        pre[k].re = suf[(size_t)d * L + k].re = (k == 0);
        pre[k].im = suf[(size_t)d * L + k].im = 0;
    }
    for (int t = 0; t < d; ++t) {
        memcpy(pre + (size_t)(t + 1) * L, pre + (size_t)t * L, sizeof(cq) * L);
        poly_mul_trunc(pre + (size_t)(t + 1) * L, U + (size_t)t * L, K);
    }
    for (int t = d - 1; t >= 0; --t) {
        memcpy(suf + (size_t)t * L, suf + (size_t)(t + 1) * L, sizeof(cq) * L);
        poly_mul_trunc(suf + (size_t)t * L, U + (size_t)t * L, K);
    }
    const int rotated = family == OR_OSC || family == OR_OSCQ || family == OR_OSCQL;
    const int nder = family == OR_OSCQL ? 3 : (family == OR_PEAK || family == OR_GAUSS || family == OR_OSCQ) ? 2 : 1;
    f128 ph = rotated ? 2 * M_PIq * (f128)params[0] : 0;
    cq rot = {cosq(ph), sinq(ph)};
    for (int t = 0; t < d; ++t) {
        cq ex[64];
        memcpy(ex, pre + (size_t)t * L, sizeof(cq) * L);
        poly_mul_trunc(ex, suf + (size_t)(t + 1) * L, K);
        for (int which = 0; which < nder; ++which) {
            cq P[64];
            memcpy(P, ex, sizeof(cq) * L);
            poly_mul_trunc(P, (which == 2 ? dU3 : which ? dU2 : dU1) + (size_t)t * L, K);
            cq s = fq_combine(&F, P);
            f128 g = rotated ? cq_mul(rot, s).re : s.re;
            if (family == OR_EXP) grad[t] = (double)g;
            else if (family == OR_OSC) grad[1 + t] = (double)g;
            else if (family == OR_OSCQ || family == OR_OSCQL) grad[1 + which * d + t] = (double)g;
            else grad[which ? d + t : t] = (double)g;
        }
    }
    if (rotated) {
        /* dQ/dw = Re(2 pi i e^{2 pi i w} S) */
        cq s = fq_combine(&F, pre + (size_t)d * L);
        cq r = cq_mul(rot, s);
        grad[0] = (double)(-2 * M_PIq * r.im);
    }
    free(U); free(dU1); free(dU2); free(dU3); free(pre); free(suf);
    fq_free(&F);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Batch driver: or_smolyak_factorised over many integrands, threads   */
/* ------------------------------------------------------------------ */
typedef struct {
    int n, nthreads, tid;
    const int *d, *q, *rule, *family;
    const int64_t *offset;
    const double *params;
    double *out;
    int rc;
} fb_job;

static void *fb_thread(void *arg)
{
    fb_job *J = (fb_job *)arg;
    for (int i = J->tid; i < J->n; i += J->nthreads) {
        double o[2];
        if (or_smolyak_factorised(J->d[i], J->q[i], J->rule[i], J->family[i], J->params + J->offset[i], o))
            J->rc = -1;
        J->out[i] = o[0];
    }
    return NULL;
}

/* Factorised values of n integrands (problem i: d[i], q[i], rule[i],
 * family[i], parameters at params + offset[i]); out[i] rounded to double. */
int or_batch_factorised(int n, const int *d, const int *q, const int *rule, const int *family,
                        const int64_t *offset, const double *params, int nthreads, double *out)
{
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    fb_job *J = calloc(nthreads, sizeof(fb_job));
    pthread_t *th = calloc(nthreads, sizeof(pthread_t));
    for (int t = 0; t < nthreads; ++t) {
        fb_job j = {n, nthreads, t, d, q, rule, family, offset, params, out, 0};
        J[t] = j;
        pthread_create(&th[t], NULL, fb_thread, &J[t]);
    }
    int rc = 0;
    for (int t = 0; t < nthreads; ++t) {
        pthread_join(th[t], NULL);
        rc |= J[t].rc;
    }
    free(J); free(th);
    return rc;
}
