// Integer layer of the Smolyak window (Section 2.1): exact counts with
// 128-bit intermediates and explicit overflow reports, the signed
// combination coefficient of (2.6), and unranking in the canonical order.
#include <algorithm>
#include <vector>

#include "sg_internal.hpp"

namespace sg {

typedef unsigned __int128 u128;
static const u128 kU64Max = (u128)UINT64_MAX;

bool binom_u64(uint64_t n, uint64_t k, uint64_t& out)
{
    if (k > n) { out = 0; return true; }
    if (k > n - k) k = n - k;
    u128 r = 1;
    for (uint64_t i = 1; i <= k; ++i) {
        // r * (n-k+i) / i is an exact binomial at every step; the product
        // fits 128 bits as long as r < 2^64 and n < 2^64
        r = r * (u128)(n - k + i) / (u128)i;
        if (r > kU64Max) return false;
    }
    out = (uint64_t)r;
    return true;
}

namespace {

// Truncated power series arithmetic on counts, saturating above 2^64-1
// with a flag (any saturated entry makes the final count an overflow).
struct SatPoly {
    std::vector<u128> c;
    bool over = false;
};

static SatPoly sat_mul(const SatPoly& a, const SatPoly& b, int K)
{
    SatPoly r;
    r.c.assign(K + 1, 0);
    r.over = a.over || b.over;
    for (int i = 0; i <= K; ++i) {
        if (a.c[i] == 0) continue;
        for (int j = 0; i + j <= K; ++j) {
            if (b.c[j] == 0) continue;
            u128 p;
            if (a.c[i] > kU64Max || b.c[j] > kU64Max) { r.over = true; p = kU64Max + 1; }
            else p = a.c[i] * b.c[j];
            if (p > kU64Max) r.over = true;
            u128 s = r.c[i + j] + std::min(p, kU64Max + 1);
            if (s > kU64Max) { r.over = true; s = kU64Max + 1; }
            r.c[i + j] = s;
        }
    }
    return r;
}

static SatPoly sat_pow(const SatPoly& base_in, uint64_t e, int K)
{
    SatPoly result;
    result.c.assign(K + 1, 0);
    result.c[0] = 1;
    SatPoly base = base_in;
    while (e) {
        if (e & 1) result = sat_mul(result, base, K);
        e >>= 1;
        if (e) base = sat_mul(base, base, K);
    }
    return result;
}

static bool add_u64(uint64_t& acc, u128 v)
{
    if (v > kU64Max) return false;
    u128 s = (u128)acc + v;
    if (s > kU64Max) return false;
    acc = (uint64_t)s;
    return true;
}

}  // namespace

sg_status counts(int d, int q, int rule, uint64_t* n_multi, uint64_t* n_rep, uint64_t* n_unique)
{
    if (d < 1 || q < d || !rule_is_known(rule)) return SG_ERR_INVALID_ARGUMENT;
    const int K = q - d;
    if (K > 60) return SG_ERR_UNSUPPORTED;
    for (int l = 1; l <= K + 1; ++l)
        if (rule_npoints(rule, l) < 1) return SG_ERR_UNSUPPORTED;
    const int e0 = std::max(0, K - d + 1);

    // multi-indices of excess e: weak compositions of e into d parts
    uint64_t m = 0;
    for (int e = e0; e <= K; ++e) {
        uint64_t c;
        if (!binom_u64((uint64_t)d - 1 + e, (uint64_t)e, c)) return SG_ERR_OVERFLOW;
        if (!add_u64(m, c)) return SG_ERR_OVERFLOW;
    }

    // n_d^q: [z^e] N(z)^d, N(z) = sum_l n_l z^(l-1), summed over the window
    SatPoly N;
    N.c.assign(K + 1, 0);
    for (int l = 1; l <= K + 1; ++l) N.c[l - 1] = (u128)rule_npoints(rule, l);
    SatPoly Nd = sat_pow(N, (uint64_t)d, K);
    uint64_t rep = 0;
    for (int e = e0; e <= K; ++e) {
        if (Nd.c[e] > kU64Max) return SG_ERR_OVERFLOW;
        if (!add_u64(rep, Nd.c[e])) return SG_ERR_OVERFLOW;
    }

    // distinct points of the union (2.4)
    uint64_t uniq = 0;
    if (rule_is_nested(rule)) {
        // a point belongs to the grid iff the levels where its coordinates
        // first appear sum to at most q: sum_{e<=K} [z^e] M(z)^d with
        // M(z) = sum_l (n_l - n_{l-1}) z^(l-1)
        SatPoly M;
        M.c.assign(K + 1, 0);
        M.c[0] = 1;
        for (int l = 2; l <= K + 1; ++l)
            M.c[l - 1] = (u128)(rule_npoints(rule, l) - rule_npoints(rule, l - 1));
        SatPoly Md = sat_pow(M, (uint64_t)d, K);
        for (int e = 0; e <= K; ++e)
            if (!add_u64(uniq, Md.c[e])) return SG_ERR_OVERFLOW;
    } else {
        // Gauss-Legendre levels share only the centre.  With c coordinates
        // at the centre and non-centre excess E (the others sit at the one
        // level owning their node), the point is reachable iff a window
        // multi-index exists: c = 0 needs K-d+1 <= E <= K; c >= 1 needs
        // E <= K, and in the paper's count (centre only in odd levels) the
        // reachable level sums step by 2, which matters only when d = 1.
        SatPoly NC;
        NC.c.assign(K + 1, 0);
        for (int l = 2; l <= K + 1; ++l) {
            long n = rule_npoints(rule, l);
            NC.c[l - 1] = (u128)(n - (n % 2));
        }
        for (int c = 0; c <= d; ++c) {
            if (c > 0 && d - c >= 0) {
                // only E <= K matter; E >= d-c (each non-centre coordinate
                // adds at least 1), so large d-c contributes nothing
                if ((long)(d - c) > (long)K) continue;
            }
            if (c == 0 && (long)d > (long)K) continue;
            SatPoly G = sat_pow(NC, (uint64_t)(d - c), K);
            uint64_t bc;
            if (!binom_u64((uint64_t)d, (uint64_t)c, bc)) {
                // binomial too big: it only matters if some G entry is non-zero
                bool any = false;
                for (int E = 0; E <= K; ++E) any = any || G.c[E] != 0;
                if (any) return SG_ERR_OVERFLOW;
                continue;
            }
            for (int E = 0; E <= K; ++E) {
                if (G.c[E] == 0) continue;
                bool ok;
                if (c == 0) {
                    ok = (E >= K - d + 1) && (E <= K);
                } else if (rule == SG_RULE_GAUSS_LEGENDRE) {
                    ok = E <= K;
                } else {
                    const long lo = (long)q - d + 1, hi = q;
                    const long s = (long)E + d;
                    ok = false;
                    for (long v = s; v <= hi; v += 2)
                        if (v >= lo) { ok = true; break; }
                }
                if (!ok) continue;
                if (G.c[E] > kU64Max) return SG_ERR_OVERFLOW;
                u128 prod = G.c[E] * (u128)bc;
                if (prod > kU64Max) return SG_ERR_OVERFLOW;
                if (!add_u64(uniq, prod)) return SG_ERR_OVERFLOW;
            }
        }
    }
    if (n_multi) *n_multi = m;
    if (n_rep) *n_rep = rep;
    if (n_unique) *n_unique = uniq;
    return SG_OK;
}

// Number of weak compositions of n into `parts` parts.
static bool weak(uint64_t n, uint64_t parts, uint64_t& out)
{
    if (parts == 0) { out = (n == 0); return true; }
    return binom_u64(n + parts - 1, n, out);
}

sg_status unrank(int d, int q, uint64_t rank, int32_t* coords, int32_t* levels, int32_t* nnz)
{
    if (d < 1 || q < d || !coords || !levels || !nnz) return SG_ERR_INVALID_ARGUMENT;
    const int K = q - d;
    if (K > 60) return SG_ERR_UNSUPPORTED;
    const int e0 = std::max(0, K - d + 1);
    // excess class
    int e = e0;
    for (;; ++e) {
        if (e > K) return SG_ERR_INVALID_ARGUMENT;
        uint64_t c;
        if (!weak((uint64_t)e, (uint64_t)d, c)) return SG_ERR_OVERFLOW;
        if (rank < c) break;
        rank -= c;
    }
    // within the class: compositions of e into positions i..d-1, in
    // decreasing lexicographic order.  Those whose first non-zero part is at
    // position j come in one block, j ascending; the block of j holds
    // W(rem-1, d-j) compositions, and the blocks of j' >= j together hold
    // W(rem, d-j) - ... ; the first position is found by binary search on
    // g(j) = W(rem, d-j) = #compositions with a_i = ... = a_{j-1} = 0.
    int i = 0, rem = e, k = 0;
    uint64_t r = rank;
    while (rem > 0) {
        uint64_t total;
        if (!weak((uint64_t)rem, (uint64_t)(d - i), total)) return SG_ERR_OVERFLOW;
        // T = total - r = number of compositions from rank r to the end
        const uint64_t T = total - r;
        // largest j in [i, d-1] with g(j) >= T
        int lo = i, hi = d - 1;
        while (lo < hi) {
            int mid = lo + (hi - lo + 1) / 2;
            uint64_t g;
            if (!weak((uint64_t)rem, (uint64_t)(d - mid), g)) return SG_ERR_OVERFLOW;
            if (g >= T) lo = mid; else hi = mid - 1;
        }
        const int j = lo;
        uint64_t gj;
        if (!weak((uint64_t)rem, (uint64_t)(d - j), gj)) return SG_ERR_OVERFLOW;
        r -= total - gj;   // skip the blocks whose first non-zero part is before j
        // a_j = a from rem down to 1; each value leaves W(rem-a, d-j-1)
        int a = rem;
        for (; a >= 1; --a) {
            uint64_t cnt;
            if (!weak((uint64_t)(rem - a), (uint64_t)(d - j - 1), cnt)) return SG_ERR_OVERFLOW;
            if (r < cnt) break;
            r -= cnt;
        }
        if (a < 1) return SG_ERR_INVALID_ARGUMENT;   // cannot happen for a valid rank
        coords[k] = j;
        levels[k] = a + 1;
        ++k;
        rem -= a;
        i = j + 1;
    }
    *nnz = k;
    return SG_OK;
}

// Frontier capacities of the point path (declared in sg_internal.hpp): over
// every ordered list of active levels (>= 2) whose excesses sum to at most K,
// the largest sum of node counts and the largest smallest two-group size.
void points_frontier_sizes(const int* n, int K, int* emax, int* cmax)
{
    // ordered lists of active levels, depth-first; sizes fit in int (P <= 6561 for K <= 8)
    int best_e = 0, best_c = 0;
    int lev[kMaxK];
    auto visit = [&](int len) {
        int E = 0, P = 1;
        for (int m = 0; m < len; ++m) {
            E += n[lev[m]];
            P *= n[lev[m]];
        }
        int c = 1 + P, pre = 1;
        for (int m = 1; m <= len; ++m) {
            pre *= n[lev[m - 1]];
            c = std::min(c, pre + P / pre);
        }
        best_e = std::max(best_e, E);
        best_c = std::max(best_c, c);
    };
    struct Rec {
        static void go(int len, int budget, int K, int* lev, const decltype(visit)& f)
        {
            if (len > 0) f(len);
            if (len == K) return;
            for (int l = 2; l - 1 <= budget; ++l) {
                lev[len] = l;
                go(len + 1, budget - (l - 1), K, lev, f);
            }
        }
    };
    Rec::go(0, K, K, lev, visit);
    *emax = best_e;
    *cmax = best_c;
}

}  // namespace sg
