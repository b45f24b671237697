// C ABI (include/sgmdi.h): contexts, plans, graph capture cache, plain
// per-integrand path, unranking, autotuning and argument validation.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <functional>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <string>
#include <tuple>
#include <vector>

#include "sg_internal.hpp"
#include "sg_oscq.hpp"

using namespace sg;

namespace {

// 1-D nodes (x - 1/2) and weights of the levels 1..K+1 of one rule, on the
// device, for the point-by-point path.
struct PointsTable {
    double* y = nullptr;
    double* w = nullptr;
    int level_off[kMaxK + 3] = {};
    int emax = 0, cmax = 0;   // frontier capacities (points_frontier_sizes)
};

// Forward schedule: target coordinates per lane and the most waves one
// problem may span.
// The default for new plans is the balanced schedule with two waves per
// SIMD (fastest on the mixed 4096-integrand workload on MI355X).
struct FwdSched {
    int cpl = 4;
    int gmax = 4;
    bool persistent = false;   // work-queue kernel instead of one workgroup per descriptor
    bool cost_scaled = false;  // cpl applies to the costliest class; cheaper classes get proportionally more
    int balanced = 2;          // > 0: equal-cost waves, this many per SIMD (pack_forward_balanced)
};

struct Records {
    std::vector<double> r64;
    std::vector<float> r32;
};

struct GraphEntry {
    const void* params;
    void* out;
    void* bound;
    void* stream;
    hipGraph_t graph;
    hipGraphExec_t exec;
};

}  // namespace

struct sg_context {
    int device = 0;
    std::string arch;                // the device's architecture name (gcnArchName)
    int n_cu = 256;                  // its compute units
    std::string last_error;
    std::map<std::pair<int, int>, std::unique_ptr<DeltaTable>> tables;
    std::map<std::pair<int, int>, std::unique_ptr<Records>> records;
    std::map<std::string, std::pair<FwdSched, bool>> tuned;   // plan shape -> (schedule, graph)
    double* one_ws = nullptr;        // scratch of the plan-free split launches (sg_integrate), counter zero
    double* noalloc = nullptr;       // the device's fixed scratch array (sg_integrate_noalloc)
    std::map<std::pair<int, int>, uint64_t*> unrank_tables;
    std::map<std::pair<int, int>, PointsTable> points_tables;   // (rule, K) -> 1-D nodes of levels 1..K+1
    double* points_ws = nullptr;                                // per-wave partial sums of the point path
    size_t points_ws_elems = 0;
    int live_plans = 0;
};

// Block (tensor-product) variant: an inner plan over the blocks, and the
// gather / combine records around it.
struct BlockedPart {
    int m = 0;                       // coordinates per block
    sg_plan* inner = nullptr;        // plan over the block sub-problems
    BlockSub* d_subs = nullptr;      // per block sub-problem (device)
    int nsub = 0;
    BlockProb* d_bprobs = nullptr;   // per integrand (device)
    double* d_params = nullptr;      // block parameters (device)
    double* d_out = nullptr;         // block values (device)
    double* d_bound = nullptr;       // block bounds (device)
    double* d_phase = nullptr;       // per sub-problem: oscillatory blocks' theta_b, sum |a_t| / 2 (device)
};

struct sg_plan {
    sg_context* ctx = nullptr;
    int precision = 0;
    int n = 0;
    std::vector<sg_problem> problems;
    ProbDev* d_probs = nullptr;
    WGDesc* d_wgs = nullptr;
    double* d_pool64 = nullptr;
    float* d_pool32 = nullptr;
    std::vector<ProbDev> probs;     // plan order (longest first)
    std::vector<double> unit_cost;  // per-coordinate cost estimate, plan order
    std::vector<double> coord_cost; // per-coordinate cost of the balanced schedule's model, plan order
    int n_cu = 0;                   // compute units of the plan's device
    double cmax = 1.0;              // largest unit cost of the plan
    int wmax = -1;                  // reverse sweep: > 0 waves cap, < 0 cost threshold (see waves_for)
    FwdSched sched;                 // forward schedule (see pack_forward)
    FwdWG* d_fwd = nullptr;         // forward workgroup descriptors
    int nfwg = 0;
    size_t fwd_capacity = 0;
    unsigned int* d_queue = nullptr; // persistent kernel: next-descriptor counter (and a spare word)
    int qgrid = 0;                  // persistent kernel: workgroups launched
    bool use_graph = false;         // replay a captured graph (else direct launch)
    bool params_disjoint = true;    // problems' parameter ranges do not overlap
    int kmax = 0;                   // largest K of the plan (kernel instantiation class)
    double* d_ws = nullptr;         // reverse-sweep workspace (sum d*K doubles), lazy
    size_t ws_elems = 0;
    int nwg = 0;
    size_t wg_capacity = 0;
    OscqDesc* d_oscq = nullptr;     // oscillatory-quadratic integrands (complex sweep)
    int noscq = 0;
    sg_plan_info info{};
    std::string tune_key;
    std::vector<GraphEntry> graphs;
    BlockedPart* blocked = nullptr;  // set for the block variant (sg_plan_create_blocked)
};

namespace {

sg_status fail(sg_context* ctx, sg_status st, const std::string& msg)
{
    if (ctx) ctx->last_error = msg;
    return st;
}

sg_status hip_fail(sg_context* ctx, hipError_t e, const char* what)
{
    std::string m = std::string(what) + ": " + hipGetErrorString(e);
    return fail(ctx, SG_ERR_DEVICE, m);
}

bool family_ok(int f)
{
    return f == SG_FAMILY_EXP_SUM || f == SG_FAMILY_OSCILLATORY || f == SG_FAMILY_PRODUCT_PEAK ||
           f == SG_FAMILY_CORNER_PEAK || f == SG_FAMILY_GAUSSIAN || f == SG_FAMILY_OSCILLATORY_QUADRATIC ||
           f == SG_FAMILY_OSCILLATORY_QUADRATIC_LINEAR;
}

// Families only the point-by-point path evaluates.
bool family_points_only(int f) { return f == SG_FAMILY_CORNER_PEAK; }

// Families on the complex sweep (k_oscq).
bool family_complex(int f)
{
    return f == SG_FAMILY_OSCILLATORY_QUADRATIC || f == SG_FAMILY_OSCILLATORY_QUADRATIC_LINEAR;
}

sg_status validate_problem(sg_context* ctx, const sg_problem& p, int idx, bool point_path = false)
{
    if (!point_path && family_points_only(p.family)) {
        char buf[200];
        snprintf(buf, sizeof buf,
                 "problem %d: family %d is evaluated by the point-by-point path only; use sg_integrate_points",
                 idx, p.family);
        return fail(ctx, SG_ERR_UNSUPPORTED, buf);
    }
    char buf[160];
    if (p.d < 1 || p.q < p.d || !rule_is_known(p.rule) || !family_ok(p.family) || p.param_offset < 0) {
        snprintf(buf, sizeof buf, "problem %d: invalid (d=%d q=%d rule=%d family=%d offset=%lld)", idx,
                 p.d, p.q, p.rule, p.family, (long long)p.param_offset);
        return fail(ctx, SG_ERR_INVALID_ARGUMENT, buf);
    }
    if (p.q - p.d > kMaxK) {
        snprintf(buf, sizeof buf, "problem %d: excess budget K=%d exceeds SG_MAX_K=%d", idx, p.q - p.d,
                 kMaxK);
        return fail(ctx, SG_ERR_UNSUPPORTED, buf);
    }
    return SG_OK;
}

const DeltaTable* get_table(sg_context* ctx, int rule, int K, sg_status& st)
{
    auto key = std::make_pair(rule, K);
    auto it = ctx->tables.find(key);
    if (it != ctx->tables.end()) return it->second.get();
    std::unique_ptr<DeltaTable> t(new DeltaTable());
    std::string err;
    if (!build_delta_table(rule, K, *t, err)) {
        st = fail(ctx, SG_ERR_INVALID_ARGUMENT, err);
        return nullptr;
    }
    const DeltaTable* r = t.get();
    ctx->tables[key] = std::move(t);
    return r;
}

const Records* get_records(sg_context* ctx, int rule, int K, sg_status& st)
{
    auto key = std::make_pair(rule, K);
    auto it = ctx->records.find(key);
    if (it != ctx->records.end()) return it->second.get();
    const DeltaTable* t = get_table(ctx, rule, K, st);
    if (!t) return nullptr;
    std::unique_ptr<Records> r(new Records());
    std::string err;
    if (!build_records(*t, r->r64, r->r32, err)) {
        st = fail(ctx, SG_ERR_INVALID_ARGUMENT, err);
        return nullptr;
    }
    const Records* out = r.get();
    ctx->records[key] = std::move(r);
    return out;
}

// Waves assigned to one problem under a schedule: sched > 0 caps every
// problem at `sched` waves (one coordinate per lane when possible); sched < 0
// gives a problem the fewest waves in {1, 2, 4} that bring one wave's work,
// ceil(d / (64 w)) * unit_cost, under -sched times the largest unit cost of
// the plan (so expensive problems are split and cheap ones are not).
int waves_for(int d, double unit_cost, int sched, double cmax)
{
    const int full = std::max(1, (d + 63) / 64);
    int w = 1;
    if (sched > 0) {
        w = std::min(full, sched);
        if (w == 3) w = 4;
    } else {
        const double T = -(double)sched * cmax;
        while (w < 4 && w < full && (double)((d + 64 * w - 1) / (64 * w)) * unit_cost > T) w *= 2;
    }
    return w;
}

// Pack problems (in plan order) into 4-wave workgroups, first fit.  A
// problem of w waves takes w consecutive slots of one workgroup.
std::vector<WGDesc> pack_workgroups(const std::vector<ProbDev>& probs, const std::vector<int>& waves)
{
    std::vector<WGDesc> wgs;
    std::vector<int> used;
    std::vector<int> open;   // indices of workgroups with free slots
    for (size_t k = 0; k < probs.size(); ++k) {
        const int w = waves[k];
        int target = -1;
        for (size_t o = 0; o < open.size(); ++o) {
            if (4 - used[open[o]] >= w) { target = open[o]; break; }
        }
        if (target < 0) {
            WGDesc e;
            std::memset(&e, 0, sizeof e);
            for (int i = 0; i < 4; ++i) { e.slot[i].prob = -1; e.slot[i].rank = 0; e.slot[i].group = 1; }
            wgs.push_back(e);
            used.push_back(0);
            target = (int)wgs.size() - 1;
            open.push_back(target);
        }
        for (int r = 0; r < w; ++r) {
            WaveSlot& sl = wgs[target].slot[used[target] + r];
            sl.p = probs[k];
            sl.p.waves = w;
            sl.prob = (int32_t)k;
            sl.rank = (int16_t)r;
            sl.group = (int16_t)w;
        }
        used[target] += w;
        if (used[target] == 4) open.erase(std::find(open.begin(), open.end(), target));
    }
    return wgs;
}

// Lanes (2^lw) and waves (group) one problem of d coordinates gets: the
// fewest lanes that keep a lane at <= cpl coordinates, or, beyond 64*cpl
// coordinates, 64 lanes on up to gmax waves of one workgroup.
void fwd_shape(int d, int cpl, int gmax, int& lw, int& group)
{
    group = 1;
    if (d > 64 * cpl) {
        lw = 6;
        const int need = (d + 64 * cpl - 1) / (64 * cpl);
        group = std::min(need <= 2 ? need : 4, gmax);
        return;
    }
    const int lanes = (d + cpl - 1) / cpl;
    lw = 2;
    while ((1 << lw) < lanes) ++lw;
}

FwdSeg seg_of(const ProbDev& p)
{
    FwdSeg g;
    g.d = p.d;
    g.out_index = p.out_index;
    g.param_offset = p.param_offset;
    return g;
}

// Forward workgroups for a schedule.  Problems are bucketed by class
// (K, rule, family) and shape; a bucket's single-wave problems (plan order,
// so longest first) fill waves side by side, multi-wave problems get their
// own waves.  Wave sets are then placed longest-first (estimated cost:
// per-lane coordinates times the class's per-coordinate cost) into 4-wave
// workgroups, first fit; the hardware dispatches workgroups in that order.
// With cost_scaled, the coordinates-per-lane target sc.cpl applies to the
// costliest class and a class of per-coordinate cost c gets
// floor(sc.cpl * cmax / c), so waves of cheap and costly classes take
// similar time.

std::vector<FwdWG> pack_forward(const std::vector<ProbDev>& probs, const std::vector<double>& unit_cost,
                                const FwdSched& sc)
{
    double cmax = 0.0;
    for (double c : unit_cost) cmax = std::max(cmax, c);
    std::map<std::tuple<int, int, int, int, int>, std::vector<int>> buckets;
    for (size_t k = 0; k < probs.size(); ++k) {
        int lw, group;
        int cpl = sc.cpl;
        if (sc.cost_scaled)
            cpl = (int)std::max(1.0, std::min(64.0, std::floor((double)sc.cpl * cmax / unit_cost[k])));
        fwd_shape(probs[k].d, cpl, sc.gmax, lw, group);
        buckets[std::make_tuple(probs[k].K, probs[k].rule, probs[k].family, lw, group)].push_back((int)k);
    }
    struct WaveSet {
        double cost;
        std::vector<FwdWave> waves;
    };
    std::vector<WaveSet> sets;
    auto base = [&](const ProbDev& pd, int lw, int group) {
        FwdWave w;
        std::memset(&w, 0, sizeof w);
        w.K = (int16_t)pd.K;
        w.rule = (int16_t)pd.rule;
        w.family = (int16_t)pd.family;
        w.lw = (int16_t)lw;
        w.group = (int16_t)group;
        w.off64 = (int32_t)pd.off64;
        w.off32 = (int32_t)pd.off32;
        for (int i = 0; i < kWaveProbs; ++i) w.seg[i].out_index = -1;
        return w;
    };
    for (auto& kv : buckets) {
        const int lw = std::get<3>(kv.first), group = std::get<4>(kv.first);
        const std::vector<int>& list = kv.second;
        if (group == 1) {
            const size_t per = (size_t)std::min(kWaveProbs, 64 >> lw);
            for (size_t i = 0; i < list.size(); i += per) {
                FwdWave w = base(probs[list[i]], lw, 1);
                int maxd = 0;
                for (size_t j = i; j < std::min(list.size(), i + per); ++j) {
                    w.seg[j - i] = seg_of(probs[list[j]]);
                    maxd = std::max(maxd, probs[list[j]].d);
                }
                w.nprob = (int16_t)(std::min(list.size(), i + per) - i);
                const int span = 1 << lw;
                const double c = unit_cost[list[i]] * (double)((maxd + span - 1) / span + 1);
                sets.push_back(WaveSet{c, std::vector<FwdWave>(1, w)});
            }
        } else {
            for (int k : list) {
                WaveSet ws;
                ws.cost = unit_cost[k] * (double)((probs[k].d + 64 * group - 1) / (64 * group) + 1);
                for (int r = 0; r < group; ++r) {
                    FwdWave w = base(probs[k], lw, group);
                    w.rank = (int16_t)r;
                    w.nprob = 1;
                    w.seg[0] = seg_of(probs[k]);
                    ws.waves.push_back(w);
                }
                sets.push_back(ws);
            }
        }
    }
    std::stable_sort(sets.begin(), sets.end(), [](const WaveSet& a, const WaveSet& b) { return a.cost > b.cost; });
    std::vector<FwdWG> wgs;
    std::vector<int> used, open;
    for (const WaveSet& ws : sets) {
        const int w = (int)ws.waves.size();
        int target = -1;
        for (int o : open)
            if (4 - used[o] >= w) { target = o; break; }
        if (target < 0) {
            FwdWG e;
            std::memset(&e, 0, sizeof e);
            for (int i = 0; i < 4; ++i) {
                e.w[i].group = 1;
                e.w[i].lw = 6;
                for (int j = 0; j < kWaveProbs; ++j) e.w[i].seg[j].out_index = -1;
            }
            wgs.push_back(e);
            used.push_back(0);
            target = (int)wgs.size() - 1;
            open.push_back(target);
        }
        for (int r = 0; r < w; ++r) wgs[target].w[used[target] + r] = ws.waves[r];
        used[target] += w;
        if (used[target] == 4) open.erase(std::find(open.begin(), open.end(), target));
    }
    return wgs;
}

// ------------------------------------------------- balanced forward schedule
// Cost model of the forward kernel on gfx950, in units of one FP32 VALU
// instruction issued per wave (FP64 operations weigh 1.65, the ratio of the
// two issue rates measured on MI355X).  Per coordinate a lane evaluates P
// node pairs and M weighted terms and multiplies one truncated polynomial;
// per wave there is a fixed cost (descriptor and parameter loads, the
// segmented reduction across lanes, the read-out) that is mostly dependency
// latency.  Calibrated against single-class plans timed on the device
// (per-coordinate costs within 10 % of the measured ones for K = 2..6,
// Clenshaw-Curtis and Gauss-Legendre, both real families).
double fwd_coord_cost(const ProbDev& p, int npairs, uint64_t macs, int precision)
{
    const int K = p.K;
    const bool series = p.family == SG_FAMILY_EXP_SUM || p.family == SG_FAMILY_OSCILLATORY;
    double pv = p.family == SG_FAMILY_GAUSSIAN ? 90.0 : p.family == SG_FAMILY_PRODUCT_PEAK ? 25.0
                : precision == SG_PREC_FP64 ? 18.0 : 7.0;
    const double mac = precision == SG_PREC_FP32_COMPENSATED ? 2.75 : 1.65;
    double c = (double)npairs * pv + (double)macs * mac + 1.65 * (double)(K * (K - 1) / 2 + K) + 4.0 * K + 31.0;
    if (p.family == SG_FAMILY_PRODUCT_PEAK) c += 40.0;            // log of the centre value
    if (K > 6 || !series) c *= 1.5;                                 // table-driven records (loads)
    // per-class corrections from per-wave timings of the kernel: the
    // Gauss-Legendre rules' wider rows at K >= 5, the Clenshaw-Curtis
    // K = 6 class's longer independent chains, the oscillatory family's
    // extra phase term
    const int rc = rule_class_of(p.rule);
    if (rc == RC_GL2 && K >= 5) c *= 1.08;
    if (rc == RC_NESTED && K == 6) c *= 0.95;
    if (p.family == SG_FAMILY_OSCILLATORY) c *= 1.03;
    // latency floor: a coordinate's dependent chain (parameter, series,
    // sums, product update) takes about this long however little work it
    // holds, with two waves sharing a SIMD (per-wave timings of the kernel)
    return c + 100.0;
}
double fwd_wave_overhead(int K, int family)
{
    // class dispatch, the first parameter load, the lane reduction (growing
    // with K), the read-out and the stores (per-wave timings of the kernel)
    return 1800.0 + 40.0 * K + (family == SG_FAMILY_OSCILLATORY ? 60.0 : 0.0);
}

// Equal-cost waves, `sc.balanced` per SIMD.  For a target wave cost T every
// problem gets the most coordinates per lane C with C * cost + overhead <= T,
// hence 2^lw lanes (or a group of up to 4 waves); problems of one class and
// shape share waves, longest first.  T is the smallest value whose waves fit
// in balanced * n_simd.  Waves then form workgroups of four of similar
// cost (a group stays inside one workgroup), and workgroups are placed so
// that every compute unit receives the same load: the hardware places
// workgroup i on compute unit i mod n_cu while all workgroups are resident,
// and each of a workgroup's four waves on its own SIMD, so a CU's SIMDs each
// take one wave of each of its workgroups.  Empty descriptors fill the
// positions no workgroup takes.
std::vector<FwdWG> pack_forward_balanced(const std::vector<ProbDev>& probs, const std::vector<double>& coord_cost,
                                         const FwdSched& sc, int n_cu, double* est_max_load)
{
    const int n_simd = 4 * n_cu;
    struct Item {
        double cost;
        std::vector<FwdWave> waves;
    };
    auto base = [&](const ProbDev& pd, int lw, int group) {
        FwdWave w;
        std::memset(&w, 0, sizeof w);
        w.K = (int16_t)pd.K;
        w.rule = (int16_t)pd.rule;
        w.family = (int16_t)pd.family;
        w.lw = (int16_t)lw;
        w.group = (int16_t)group;
        w.off64 = (int32_t)pd.off64;
        w.off32 = (int32_t)pd.off32;
        for (int i = 0; i < kWaveProbs; ++i) w.seg[i].out_index = -1;
        return w;
    };
    auto build = [&](double T, std::vector<Item>& items) {
        items.clear();
        std::map<std::tuple<int, int, int, int, int>, std::vector<int>> buckets;
        for (size_t k = 0; k < probs.size(); ++k) {
            const ProbDev& pd = probs[k];
            const double o = fwd_wave_overhead(pd.K, pd.family);
            const int C = (int)std::max(1.0, std::min(4096.0, std::floor((T - o) / coord_cost[k])));
            const int lanes = (pd.d + C - 1) / C;
            int lw = 2, group = 1;
            if (lanes > 64) {
                lw = 6;
                group = (lanes + 63) / 64;
                group = group <= 1 ? 1 : group <= 2 ? 2 : 4;
                group = std::min(group, sc.gmax);
            } else {
                while ((1 << lw) < lanes) ++lw;
            }
            buckets[std::make_tuple(pd.K, pd.rule, pd.family, lw, group)].push_back((int)k);
        }
        for (auto& kv : buckets) {
            const int lw = std::get<3>(kv.first), group = std::get<4>(kv.first);
            std::vector<int> list = kv.second;
            std::stable_sort(list.begin(), list.end(), [&](int a, int b) { return probs[a].d > probs[b].d; });
            const ProbDev& p0 = probs[list[0]];
            const double o = fwd_wave_overhead(p0.K, p0.family);
            if (group == 1) {
                const size_t per = (size_t)std::min(kWaveProbs, 64 >> lw);
                for (size_t i = 0; i < list.size(); i += per) {
                    FwdWave w = base(probs[list[i]], lw, 1);
                    int maxd = 0;
                    for (size_t j = i; j < std::min(list.size(), i + per); ++j) {
                        w.seg[j - i] = seg_of(probs[list[j]]);
                        maxd = std::max(maxd, probs[list[j]].d);
                    }
                    w.nprob = (int16_t)(std::min(list.size(), i + per) - i);
                    const int span = 1 << lw;
                    items.push_back(Item{(double)((maxd + span - 1) / span) * coord_cost[list[i]] + o,
                                         std::vector<FwdWave>(1, w)});
                }
            } else {
                for (int k : list) {
                    Item it;
                    it.cost = (double)((probs[k].d + 64 * group - 1) / (64 * group)) * coord_cost[k] + o +
                              200.0 * group;
                    for (int r = 0; r < group; ++r) {
                        FwdWave w = base(probs[k], lw, group);
                        w.rank = (int16_t)r;
                        w.nprob = 1;
                        w.seg[0] = seg_of(probs[k]);
                        it.waves.push_back(w);
                    }
                    items.push_back(it);
                }
            }
        }
    };
    auto nwaves = [](const std::vector<Item>& items) {
        size_t n = 0;
        for (const Item& it : items) n += it.waves.size();
        return n;
    };
    // smallest T (bisection on a log scale) whose waves fit
    std::vector<Item> items;
    const size_t cap = (size_t)std::max(1, sc.balanced) * (size_t)n_simd;
    double lo = 1.0, hi = 1.0;
    for (;;) {
        build(hi, items);
        if (nwaves(items) <= cap || hi > 1e12) break;
        lo = hi;
        hi *= 2.0;
    }
    for (int it = 0; it < 40 && hi > lo * 1.001; ++it) {
        const double mid = std::sqrt(lo * hi);
        build(mid, items);
        if (nwaves(items) <= cap) hi = mid;
        else lo = mid;
    }
    build(hi, items);
    // workgroups: items longest first, first fit into 4-wave workgroups
    std::stable_sort(items.begin(), items.end(), [](const Item& a, const Item& b) { return a.cost > b.cost; });
    struct WG {
        FwdWG desc;
        int used = 0;
        double cost[4] = {0, 0, 0, 0};
    };
    std::vector<WG> wgs;
    std::vector<int> open;
    for (const Item& it : items) {
        const int w = (int)it.waves.size();
        int target = -1;
        for (int o : open)
            if (4 - wgs[o].used >= w) { target = o; break; }
        if (target < 0) {
            WG e;
            std::memset(&e.desc, 0, sizeof e.desc);
            for (int i = 0; i < 4; ++i) {
                e.desc.w[i].group = 1;
                e.desc.w[i].lw = 6;
                for (int j = 0; j < kWaveProbs; ++j) e.desc.w[i].seg[j].out_index = -1;
            }
            wgs.push_back(e);
            target = (int)wgs.size() - 1;
            open.push_back(target);
        }
        WG& g = wgs[target];
        for (int r = 0; r < w; ++r) {
            g.desc.w[g.used + r] = it.waves[r];
            g.cost[g.used + r] = it.cost;
        }
        g.used += w;
        if (g.used == 4) open.erase(std::find(open.begin(), open.end(), target));
    }
    // placement: workgroups longest first, each to the compute unit with the
    // least load (its SIMDs' loads, the workgroup's costliest wave joining
    // the least-loaded SIMD) among those with the fewest workgroups
    std::vector<int> wg_order(wgs.size());
    for (size_t i = 0; i < wgs.size(); ++i) wg_order[i] = (int)i;
    auto wg_cost = [&](int i) { return wgs[i].cost[0] + wgs[i].cost[1] + wgs[i].cost[2] + wgs[i].cost[3]; };
    std::stable_sort(wg_order.begin(), wg_order.end(), [&](int a, int b) { return wg_cost(a) > wg_cost(b); });
    std::vector<std::array<double, 4>> simd(n_cu, std::array<double, 4>{0, 0, 0, 0});
    std::vector<int> count(n_cu, 0);
    std::vector<int> pos(wgs.size(), -1);
    const int rounds = (int)((wgs.size() + n_cu - 1) / n_cu);
    for (int i : wg_order) {
        int best = -1;
        double bl = 0.0;
        for (int c = 0; c < n_cu; ++c) {
            if (count[c] >= rounds) continue;
            const double l = simd[c][0] + simd[c][1] + simd[c][2] + simd[c][3];
            if (best < 0 || l < bl) { best = c; bl = l; }
        }
        std::array<double, 4> wc{wgs[i].cost[0], wgs[i].cost[1], wgs[i].cost[2], wgs[i].cost[3]};
        std::sort(wc.begin(), wc.end(), std::greater<double>());
        std::array<int, 4> idx{0, 1, 2, 3};
        std::sort(idx.begin(), idx.end(), [&](int a, int b) { return simd[best][a] < simd[best][b]; });
        for (int k = 0; k < 4; ++k) simd[best][idx[k]] += wc[k];
        pos[i] = best + n_cu * count[best];
        count[best]++;
    }
    int npos = 0;
    for (int p : pos) npos = std::max(npos, p + 1);
    std::vector<FwdWG> out((size_t)npos);
    for (FwdWG& e : out) {
        std::memset(&e, 0, sizeof e);
        for (int i = 0; i < 4; ++i) {
            e.w[i].group = 1;
            e.w[i].lw = 6;
            for (int j = 0; j < kWaveProbs; ++j) e.w[i].seg[j].out_index = -1;
        }
    }
    for (size_t i = 0; i < wgs.size(); ++i) out[(size_t)pos[i]] = wgs[i].desc;
    if (est_max_load) {
        double m = 0.0;
        for (auto& a : simd) m = std::max(m, std::max(std::max(a[0], a[1]), std::max(a[2], a[3])));
        *est_max_load = m;
    }
    return out;
}

uint64_t macs_of(const DeltaTable& t)
{
    uint64_t m = 0;
    for (int L = 2; L <= t.K + 1; ++L) {
        const uint64_t np = (uint64_t)(t.level_begin[L + 1] - t.level_begin[L]);
        const uint64_t ne = t.nested ? (uint64_t)(t.K - L + 2) : (uint64_t)(L <= t.K ? 2 : 1);
        m += np * ne;
    }
    return m;
}

uint64_t sat_add(uint64_t a, uint64_t b)
{
    return a > UINT64_MAX - b ? UINT64_MAX : a + b;
}

uint64_t sat_mul(uint64_t a, uint64_t b)
{
    if (a == 0 || b == 0) return 0;
    return a > UINT64_MAX / b ? UINT64_MAX : a * b;
}

template <class T>
sg_status upload(sg_context* ctx, T** dst, const T* src, size_t n)
{
    const size_t bytes = std::max<size_t>(1, n) * sizeof(T);
    hipError_t e = hipMalloc((void**)dst, bytes);
    if (e != hipSuccess) return fail(ctx, SG_ERR_OUT_OF_MEMORY, std::string("hipMalloc: ") + hipGetErrorString(e));
    if (n) {
        e = hipMemcpy(*dst, src, n * sizeof(T), hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            (void)hipFree(*dst);
            *dst = nullptr;
            return hip_fail(ctx, e, "hipMemcpy");
        }
    }
    return SG_OK;
}

void destroy_graphs(sg_plan* p)
{
    for (GraphEntry& g : p->graphs) {
        (void)hipGraphExecDestroy(g.exec);
        (void)hipGraphDestroy(g.graph);
    }
    p->graphs.clear();
}

bool graphs_enabled()
{
    const char* v = std::getenv("SGMDI_NO_GRAPH");
    return !(v && v[0] && v[0] != '0');
}

}  // namespace

extern "C" {

const char* sg_status_string(sg_status s)
{
    switch (s) {
    case SG_OK: return "ok";
    case SG_ERR_INVALID_ARGUMENT: return "invalid argument";
    case SG_ERR_UNSUPPORTED: return "unsupported";
    case SG_ERR_OVERFLOW: return "count overflows 64 bits";
    case SG_ERR_OUT_OF_MEMORY: return "out of memory";
    case SG_ERR_DEVICE: return "device error";
    case SG_ERR_CAPTURE: return "graph capture failed";
    }
    return "unknown status";
}

const char* sg_last_error(const sg_context* ctx)
{
    return ctx ? ctx->last_error.c_str() : "no context";
}

sg_status sg_context_create(sg_context** ctx)
{
    if (!ctx) return SG_ERR_INVALID_ARGUMENT;
    *ctx = nullptr;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return SG_ERR_DEVICE;
    sg_context* c = new (std::nothrow) sg_context();
    if (!c) return SG_ERR_OUT_OF_MEMORY;
    c->device = dev;
    hipDeviceProp_t prop;
    std::memset(&prop, 0, sizeof prop);
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) {
        delete c;
        return SG_ERR_DEVICE;
    }
    prop.gcnArchName[sizeof prop.gcnArchName - 1] = 0;
    c->arch = prop.gcnArchName;
    if (prop.multiProcessorCount > 0) c->n_cu = prop.multiProcessorCount;
    // set-up of the allocation-free path: the address of this device's fixed
    // scratch array (looked up once per device)
    const int rc = noalloc_scratch(&c->noalloc);
    if (rc != 0) {
        delete c;
        return SG_ERR_DEVICE;
    }
    *ctx = c;
    return SG_OK;
}

sg_status sg_context_destroy(sg_context* ctx)
{
    if (!ctx) return SG_OK;
    (void)hipFree(ctx->one_ws);
    for (auto& kv : ctx->unrank_tables) (void)hipFree(kv.second);
    for (auto& kv : ctx->points_tables) {
        (void)hipFree(kv.second.y);
        (void)hipFree(kv.second.w);
    }
    (void)hipFree(ctx->points_ws);
    delete ctx;
    return SG_OK;
}

sg_status sg_counts(int32_t d, int32_t q, int32_t rule, uint64_t* n_multi, uint64_t* n_points_rep,
                    uint64_t* n_points_unique)
{
    return counts(d, q, rule, n_multi, n_points_rep, n_points_unique);
}

sg_status sg_rule_table(int32_t rule, int32_t level, double* x, double* w, int32_t* n)
{
    if (!rule_is_known(rule) || level < 1) return SG_ERR_INVALID_ARGUMENT;
    const long np = rule_npoints(rule, level);
    if (np < 1) return SG_ERR_UNSUPPORTED;
    if (n) *n = (int32_t)np;
    if (!x && !w) return SG_OK;
    if (!x || !w) return SG_ERR_INVALID_ARGUMENT;
    std::vector<long double> xs, ws;
    if (!rule_nodes(rule, level, xs, ws)) return SG_ERR_UNSUPPORTED;
    for (long j = 0; j < np; ++j) {
        x[j] = (double)xs[j];
        w[j] = (double)ws[j];
    }
    return SG_OK;
}

sg_status sg_coefficient(int32_t d, int32_t q, int32_t e, int64_t* coef)
{
    if (d < 1 || q < d || !coef) return SG_ERR_INVALID_ARGUMENT;
    const int K = q - d;
    if (e < std::max(0, K - d + 1) || e > K) { *coef = 0; return SG_OK; }
    uint64_t c;
    if (!binom_u64((uint64_t)d - 1, (uint64_t)(K - e), c) || c > (uint64_t)INT64_MAX) return SG_ERR_OVERFLOW;
    *coef = ((K - e) % 2) ? -(int64_t)c : (int64_t)c;
    return SG_OK;
}

sg_status sg_unrank(int32_t d, int32_t q, uint64_t rank, int32_t* coords, int32_t* levels, int32_t* nnz)
{
    if (d < 1 || q < d) return SG_ERR_INVALID_ARGUMENT;
    uint64_t m;
    sg_status st = counts(d, q, SG_RULE_CLENSHAW_CURTIS, &m, nullptr, nullptr);
    if (st == SG_ERR_OVERFLOW) {
        // the multi-index count alone may still fit; recount it directly
        const int K = q - d;
        m = 0;
        for (int e = std::max(0, K - d + 1); e <= K; ++e) {
            uint64_t c;
            if (!binom_u64((uint64_t)d - 1 + e, (uint64_t)e, c) || m > UINT64_MAX - c) return SG_ERR_OVERFLOW;
            m += c;
        }
    } else if (st != SG_OK) {
        return st;
    }
    if (rank >= m) return SG_ERR_INVALID_ARGUMENT;
    return unrank(d, q, rank, coords, levels, nnz);
}

// Weak-composition counts W[n][parts] (n <= K, parts <= d) on the device
// (cached per (d, q)) and the window's multi-index count.
static sg_status window_table(sg_context* ctx, int d, int q, uint64_t** dW, uint64_t* n_multi)
{
    const int K = q - d;
    std::vector<uint64_t> W((size_t)(K + 1) * (d + 1), 0);
    for (int nn = 0; nn <= K; ++nn)
        for (int parts = 0; parts <= d; ++parts) {
            uint64_t v;
            if (parts == 0) v = (nn == 0);
            else if (!binom_u64((uint64_t)nn + parts - 1, (uint64_t)nn, v))
                return fail(ctx, SG_ERR_OVERFLOW, "window not countable in 64 bits");
            W[(size_t)nn * (d + 1) + parts] = v;
        }
    uint64_t m = 0;
    for (int e = std::max(0, K - d + 1); e <= K; ++e) {
        const uint64_t c = W[(size_t)e * (d + 1) + d];
        if (m > UINT64_MAX - c) return fail(ctx, SG_ERR_OVERFLOW, "window not countable in 64 bits");
        m += c;
    }
    *n_multi = m;
    auto key = std::make_pair(d, q);
    auto it = ctx->unrank_tables.find(key);
    if (it == ctx->unrank_tables.end()) {
        uint64_t* p = nullptr;
        sg_status st = upload(ctx, &p, W.data(), W.size());
        if (st != SG_OK) return st;
        ctx->unrank_tables[key] = p;
        *dW = p;
    } else {
        *dW = it->second;
    }
    return SG_OK;
}

sg_status sg_unrank_device(sg_context* ctx, int32_t d, int32_t q, uint64_t rank0, uint64_t count,
                           int32_t max_nnz, int32_t* coords_dev, int32_t* levels_dev, int32_t* nnz_dev,
                           void* stream)
{
    if (!ctx) return SG_ERR_INVALID_ARGUMENT;
    if (d < 1 || q < d || !coords_dev || !levels_dev || !nnz_dev)
        return fail(ctx, SG_ERR_INVALID_ARGUMENT, "sg_unrank_device: bad d/q or NULL output");
    const int K = q - d;
    if (K > 60) return fail(ctx, SG_ERR_UNSUPPORTED, "K > 60");
    if (max_nnz < std::max(1, K)) return fail(ctx, SG_ERR_INVALID_ARGUMENT, "max_nnz < K");
    uint64_t* dW = nullptr;
    uint64_t m = 0;
    sg_status st = window_table(ctx, d, q, &dW, &m);
    if (st != SG_OK) return st;
    if (count == 0) return SG_OK;
    if (rank0 >= m || count > m - rank0) return fail(ctx, SG_ERR_INVALID_ARGUMENT, "rank range beyond the window");
    const int rc = launch_unrank(d, q, rank0, count, max_nnz, dW, K + 1, coords_dev, levels_dev, nnz_dev, stream);
    if (rc != 0) return hip_fail(ctx, (hipError_t)rc, "unrank launch");
    return SG_OK;
}

sg_status sg_integrate_points(sg_context* ctx, const sg_problem* problem, const double* params_dev,
                              double* out_dev, double* bound_dev, uint64_t max_points, void* stream)
{
    if (!ctx) return SG_ERR_INVALID_ARGUMENT;
    if (!problem || !params_dev || !out_dev) return fail(ctx, SG_ERR_INVALID_ARGUMENT, "NULL argument");
    sg_status st = validate_problem(ctx, *problem, 0, true);
    if (st != SG_OK) return st;
    const int d = problem->d, q = problem->q, K = q - d, rule = problem->rule;
    uint64_t npts = 0;
    st = counts(d, q, rule, nullptr, &npts, nullptr);
    if (st != SG_OK) return fail(ctx, st, "point count not representable in 64 bits");
    if (max_points && npts > max_points)
        return fail(ctx, SG_ERR_UNSUPPORTED, "more points than max_points (" + std::to_string(npts) + ")");
    uint64_t* dW = nullptr;
    uint64_t n_multi = 0;
    if ((st = window_table(ctx, d, q, &dW, &n_multi)) != SG_OK) return st;
    // 1-D nodes of levels 1..K+1
    auto key = std::make_pair(rule, K);
    auto it = ctx->points_tables.find(key);
    if (it == ctx->points_tables.end()) {
        PointsTable pt;
        std::vector<double> ys, ws;
        std::vector<long double> x, w;
        pt.level_off[0] = pt.level_off[1] = 0;
        for (int l = 1; l <= K + 1; ++l) {
            if (!rule_nodes(rule, l, x, w)) return fail(ctx, SG_ERR_UNSUPPORTED, "rule construction failed");
            for (size_t j = 0; j < x.size(); ++j) {
                ys.push_back((double)(x[j] - 0.5L));
                ws.push_back((double)w[j]);
            }
            pt.level_off[l + 1] = (int)ys.size();
        }
        for (int l = K + 2; l < kMaxK + 3; ++l) pt.level_off[l] = (int)ys.size();
        int nl[kMaxK + 3] = {};
        for (int l = 1; l <= K + 1; ++l) nl[l] = pt.level_off[l + 1] - pt.level_off[l];
        points_frontier_sizes(nl, K, &pt.emax, &pt.cmax);
        if ((st = upload(ctx, &pt.y, ys.data(), ys.size())) != SG_OK) return st;
        if ((st = upload(ctx, &pt.w, ws.data(), ws.size())) != SG_OK) {
            (void)hipFree(pt.y);
            return st;
        }
        it = ctx->points_tables.emplace(key, pt).first;
    }
    // grid: every wave gets at least one chunk of 64 ranks; at most 2048 workgroups
    const uint64_t nchunks = (n_multi + 63) / 64;
    const int grid = (int)std::max<uint64_t>(1, std::min<uint64_t>(2048, (nchunks + 3) / 4));
    const size_t ws_need = (size_t)grid * 4 * 3;
    if (ws_need > ctx->points_ws_elems) {
        (void)hipFree(ctx->points_ws);
        ctx->points_ws = nullptr;
        ctx->points_ws_elems = 0;
        hipError_t e = hipMalloc((void**)&ctx->points_ws, ws_need * sizeof(double));
        if (e != hipSuccess) return fail(ctx, SG_ERR_OUT_OF_MEMORY, std::string("hipMalloc: ") + hipGetErrorString(e));
        ctx->points_ws_elems = ws_need;
    }
    PointsLaunch L;
    L.d = d;
    L.K = K;
    L.e0 = std::max(0, K - d + 1);
    L.grid = grid;
    L.n_multi = n_multi;
    L.W = dW;
    L.node_y = it->second.y;
    L.node_w = it->second.w;
    for (int i = 0; i < kMaxK + 3; ++i) L.level_off[i] = it->second.level_off[i];
    L.emax = it->second.emax;
    L.cmax = it->second.cmax;
    for (int e = 0; e <= kMaxK; ++e) {
        // (-1)^(K-e) C(d-1, K-e), exact in long double up to 2^64, rounded once
        long double c = 0.0L;
        if (e <= K && K - e <= d - 1) {
            c = 1.0L;
            for (int j = 1; j <= K - e; ++j) c = c * (long double)(d - 1 - (K - e) + j) / (long double)j;
            if ((K - e) % 2) c = -c;
        }
        L.coef[e] = (double)c;
    }
    L.params = params_dev;
    L.partial = ctx->points_ws;
    L.out = out_dev;
    L.bound = bound_dev;
    const int rc = launch_points(problem->family, L, stream);
    if (rc != 0) return hip_fail(ctx, (hipError_t)rc, "point path launch");
    return SG_OK;
}

static sg_status plan_repack(sg_plan* p, const FwdSched& sc);
static void plan_free(sg_plan* p);

// Autotune key of a plan: precision, problem count and a 64-bit FNV-1a hash
// of the sorted (d, K, rule, family) list, so that only plans of the same
// shape share a tuned schedule.
static std::string tune_key(int precision, const sg_problem* problems, int n)
{
    std::vector<std::array<int32_t, 4>> cls((size_t)n);
    for (int i = 0; i < n; ++i)
        cls[(size_t)i] = {problems[i].d, problems[i].q - problems[i].d, problems[i].rule, problems[i].family};
    std::sort(cls.begin(), cls.end());
    uint64_t h = 1469598103934665603ull;
    for (const auto& c : cls)
        for (int32_t v : c)
            for (int b = 0; b < 4; ++b) {
                h ^= (uint64_t)(((uint32_t)v >> (8 * b)) & 0xffu);
                h *= 1099511628211ull;
            }
    char key[64];
    std::snprintf(key, sizeof key, "p%d_n%d_%016llx", precision, n, (unsigned long long)h);
    return key;
}
// Owner of a plan under construction: a failed creation releases whatever
// it had allocated.
struct PlanFree {
    void operator()(sg_plan* p) const { plan_free(p); }
};
using PlanOwner = std::unique_ptr<sg_plan, PlanFree>;

sg_status sg_plan_create(sg_context* ctx, const sg_problem* problems, int32_t n, int32_t precision,
                         sg_plan** plan)
{
    if (!ctx || !plan) return SG_ERR_INVALID_ARGUMENT;
    *plan = nullptr;
    if (!problems || n < 1) return fail(ctx, SG_ERR_INVALID_ARGUMENT, "empty problem list");
    if (precision != SG_PREC_FP64 && precision != SG_PREC_FP32_COMPENSATED && precision != SG_PREC_FP32_FP64_SUM)
        return fail(ctx, SG_ERR_INVALID_ARGUMENT, "unknown precision");
    for (int i = 0; i < n; ++i) {
        sg_status st = validate_problem(ctx, problems[i], i);
        if (st != SG_OK) return st;
    }
    PlanOwner p(new sg_plan());
    p->ctx = ctx;
    p->precision = precision;
    p->n = n;
    p->problems.assign(problems, problems + n);

    // record tables, one per distinct (rule, K), in two pools
    std::map<std::pair<int, int>, std::pair<int64_t, int64_t>> toff;
    std::vector<double> p64;
    std::vector<float> p32;
    std::vector<const DeltaTable*> ptab(n);
    for (int i = 0; i < n; ++i) {
        auto key = std::make_pair(problems[i].rule, problems[i].q - problems[i].d);
        sg_status st = SG_OK;
        const DeltaTable* t = get_table(ctx, key.first, key.second, st);
        if (!t) return st;
        ptab[i] = t;
        if (toff.count(key)) continue;
        const Records* r = get_records(ctx, key.first, key.second, st);
        if (!r) return st;
        toff[key] = std::make_pair((int64_t)p64.size(), (int64_t)p32.size());
        p64.insert(p64.end(), r->r64.begin(), r->r64.end());
        p32.insert(p32.end(), r->r32.begin(), r->r32.end());
        while (p64.size() % 8) p64.push_back(0.0);     // 64-byte aligned tables
        while (p32.size() % 16) p32.push_back(0.0f);
    }

    // longest-processing-time order
    std::vector<double> cost(n);
    sg_plan_info info{};
    bool has_gauss = false;
    for (int i = 0; i < n; ++i) {
        const DeltaTable& t = *ptab[i];
        const uint64_t d = (uint64_t)problems[i].d;
        const uint64_t K = (uint64_t)t.K;
        const uint64_t macs = macs_of(t);
        cost[i] = (double)d * (8.0 * t.npairs + 2.0 * (double)macs + (double)(K * K));
        uint64_t nrep = 0;
        sg_status st = counts(problems[i].d, problems[i].q, problems[i].rule, nullptr, &nrep, nullptr);
        info.effective_points = sat_add(info.effective_points, st == SG_OK ? nrep : UINT64_MAX);
        info.units = sat_add(info.units, d);
        info.pair_evals = sat_add(info.pair_evals, sat_mul(d, (uint64_t)t.npairs));
        info.macs = sat_add(info.macs, sat_mul(d, macs));
        info.merge_flops = sat_add(info.merge_flops, sat_mul(d, K * K));
        if (family_complex(problems[i].family)) continue;   // its own kernel
        p->kmax = std::max(p->kmax, (int)K);
        if (problems[i].family == SG_FAMILY_GAUSSIAN) has_gauss = true;
    }
    if (has_gauss) p->kmax = kKmaxGauss;   // the forward kernels built with the gaussian family
    // the sweep kernels' problems in longest-first order; the oscillatory
    // quadratic (complex surpluses) to its own kernel, one workgroup each
    std::vector<int> order;
    std::vector<OscqDesc> oscq;
    for (int i = 0; i < n; ++i) {
        if (!family_complex(problems[i].family)) {
            order.push_back(i);
            continue;
        }
        OscqDesc q;
        q.ws_off = 0;
        const auto& qo = toff[std::make_pair(problems[i].rule, problems[i].q - problems[i].d)];
        q.off64 = qo.first;
        q.off32 = qo.second;
        q.param_offset = problems[i].param_offset;
        q.d = problems[i].d;
        q.K = problems[i].q - problems[i].d;
        q.rule = problems[i].rule;
        q.out_index = i;
        q.lin = problems[i].family == SG_FAMILY_OSCILLATORY_QUADRATIC_LINEAR ? 1 : 0;
        q.reserved = 0;
        oscq.push_back(q);
    }
    const int nr = (int)order.size();
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost[a] > cost[b]; });
    p->probs.resize(nr);
    p->unit_cost.resize(nr);
    p->coord_cost.resize(nr);
    for (int k = 0; k < nr; ++k) {
        const int i = order[k];
        p->unit_cost[k] = cost[i] / (double)problems[i].d;
        p->cmax = std::max(p->cmax, p->unit_cost[k]);
        ProbDev& r = p->probs[k];
        const int K = problems[i].q - problems[i].d;
        r.d = problems[i].d;
        r.K = K;
        r.family = problems[i].family;
        r.rule = problems[i].rule;
        r.param_offset = problems[i].param_offset;
        const auto& o = toff[std::make_pair(problems[i].rule, K)];
        r.off64 = o.first;
        r.off32 = o.second;
        r.out_index = i;
        r.waves = 0;
        p->coord_cost[k] = fwd_coord_cost(r, ptab[i]->npairs, macs_of(*ptab[i]), precision);
        r.ws_off = (int64_t)p->ws_elems;
        p->ws_elems += (size_t)r.d * (size_t)(K > 0 ? K : 1);
    }
    // reverse sweep of the oscillatory quadratic: d complex surpluses each
    for (OscqDesc& q : oscq) {
        q.ws_off = (int64_t)p->ws_elems;
        p->ws_elems += (size_t)q.d * (size_t)(2 * (q.K > 0 ? q.K : 1));
    }
    {
        // parameter ranges must be disjoint for the reverse sweep to write them
        std::vector<std::pair<int64_t, int64_t>> rg(n);
        for (int i = 0; i < n; ++i) {
            const int f = problems[i].family;
            const int64_t d = problems[i].d;
            const int64_t len = f == SG_FAMILY_EXP_SUM ? d
                                : f == SG_FAMILY_OSCILLATORY ? d + 1
                                : f == SG_FAMILY_OSCILLATORY_QUADRATIC ? 2 * d + 1
                                : f == SG_FAMILY_OSCILLATORY_QUADRATIC_LINEAR ? 3 * d + 1 : 2 * d;
            rg[i] = std::make_pair(problems[i].param_offset, problems[i].param_offset + len);
        }
        std::sort(rg.begin(), rg.end());
        for (int i = 1; i < n; ++i)
            if (rg[i].first < rg[i - 1].second) p->params_disjoint = false;
    }

    p->tune_key = tune_key(precision, problems, n);
    auto tk = ctx->tuned.find(p->tune_key);
    if (tk != ctx->tuned.end()) {
        p->sched = tk->second.first;
        p->use_graph = tk->second.second;
    }
    if (const char* fs = std::getenv("SGMDI_SCHED")) {   // profiling override: "cpl,gmax[,persistent[,cost_scaled]]"
        int c = 0, g = 0, q = 0, cs = 0;
        const int nf = std::sscanf(fs, "%d,%d,%d,%d", &c, &g, &q, &cs);
        if (nf >= 2 && c >= 1 && c <= 64 && (g == 1 || g == 2 || g == 4)) {
            p->sched.balanced = 0;
            p->sched.cpl = c;
            p->sched.gmax = g;
            p->sched.persistent = nf >= 3 && q == 1;
            p->sched.cost_scaled = nf >= 4 && cs == 1;
        }
    }
    p->n_cu = ctx->n_cu;
    // reverse sweep: one problem per wave slot, cost-threshold schedule
    std::vector<int> wv(nr);
    for (int k = 0; k < nr; ++k) wv[k] = waves_for(p->probs[k].d, p->unit_cost[k], p->wmax, p->cmax);
    std::vector<WGDesc> wgs = pack_workgroups(p->probs, wv);
    for (int k = 0; k < nr; ++k) p->probs[k].waves = wv[k];
    p->nwg = (int)wgs.size();
    info.block_threads = 256;
    info.graph = p->use_graph ? 1 : 0;
    p->info = info;

    sg_status st;
    if ((st = upload(ctx, &p->d_probs, p->probs.data(), p->probs.size())) != SG_OK) return st;
    if ((st = upload(ctx, &p->d_wgs, wgs.data(), wgs.size())) != SG_OK) return st;
    p->wg_capacity = wgs.size();
    {
        hipError_t e = hipMalloc((void**)&p->d_queue, 2 * sizeof(unsigned int));
        if (e != hipSuccess) return fail(ctx, SG_ERR_OUT_OF_MEMORY, std::string("hipMalloc: ") + hipGetErrorString(e));
    }
    // forward sweep: class-uniform waves, problems side by side
    if ((st = plan_repack(p.get(), p->sched)) != SG_OK) return st;
    if ((st = upload(ctx, &p->d_pool64, p64.data(), p64.size())) != SG_OK) return st;
    if ((st = upload(ctx, &p->d_pool32, p32.data(), p32.size())) != SG_OK) return st;
    if (!oscq.empty()) {
        if ((st = upload(ctx, &p->d_oscq, oscq.data(), oscq.size())) != SG_OK) return st;
        p->noscq = (int)oscq.size();
        p->info.fp64_complex = p->noscq;
    }
    ctx->live_plans++;
    *plan = p.release();
    return SG_OK;
}

static sg_status plan_launch(sg_plan* p, const double* params, double* out, double* bound, void* stream)
{
    const int rc = launch_forward(p->precision, p->kmax, p->nfwg, p->d_fwd, p->sched.persistent ? p->d_queue : nullptr,
                                  p->qgrid, p->d_pool64, p->d_pool32, params, out, bound, stream);
    if (rc != 0) return hip_fail(p->ctx, (hipError_t)rc, "forward launch");
    if (p->noscq) {
        const int rq = launch_oscq_batch(p->precision, p->noscq, p->d_oscq, p->d_pool64, p->d_pool32, params, out,
                                         bound, stream);
        if (rq != 0) return hip_fail(p->ctx, (hipError_t)rq, "oscillatory-quadratic launch");
    }
    return SG_OK;
}

// Re-pack the plan's forward workgroups for another schedule.
static sg_status plan_repack(sg_plan* p, const FwdSched& sc_in)
{
    FwdSched sc = sc_in;
    if (sc.balanced > 0) sc.persistent = false;   // placement relies on hardware dispatch order
    std::vector<FwdWG> fwd = sc.balanced > 0 ? pack_forward_balanced(p->probs, p->coord_cost, sc, p->n_cu, nullptr)
                                             : pack_forward(p->probs, p->unit_cost, sc);
    // the workgroup-level flag the kernel reads instead of the four group sizes
    for (FwdWG& e : fwd) {
        e.w[0].grouped = 0;
        for (int i = 0; i < 4; ++i)
            if (e.w[i].group > 1) e.w[0].grouped = 1;
    }
    if (fwd.size() > p->fwd_capacity) {
        // the new buffer first: on failure the plan keeps its schedule
        FwdWG* grown = nullptr;
        sg_status st = upload(p->ctx, &grown, fwd.data(), fwd.size());
        if (st != SG_OK) return st;
        (void)hipFree(p->d_fwd);
        p->d_fwd = grown;
        p->fwd_capacity = fwd.size();
    } else {
        hipError_t e = hipMemcpy(p->d_fwd, fwd.data(), fwd.size() * sizeof(FwdWG), hipMemcpyHostToDevice);
        if (e != hipSuccess) return hip_fail(p->ctx, e, "hipMemcpy");
    }
    p->sched = sc;
    p->nfwg = (int)fwd.size();
    const int cap = forward_capacity(p->precision, p->kmax);
    if (cap <= 0) p->sched.persistent = false;
    p->qgrid = std::max(1, std::min(p->nfwg, cap));
    if (p->sched.persistent) {
        // counters start at zero; each launch leaves them at zero
        hipError_t e = hipMemset(p->d_queue, 0, 2 * sizeof(unsigned int));
        if (e != hipSuccess) return hip_fail(p->ctx, e, "hipMemset");
    }
    p->info.grid_blocks = p->sched.persistent ? p->qgrid : p->nfwg;
    p->info.coords_per_lane = sc.cpl;
    p->info.max_group = sc.gmax;
    p->info.persistent = p->sched.persistent ? 1 : 0;
    p->info.cost_scaled = sc.cost_scaled ? 1 : 0;
    p->info.balanced = sc.balanced;
    return SG_OK;
}

static sg_status blocked_execute(sg_plan* p, const double* params_dev, double* out_dev, double* bound_dev,
                                 void* stream);

// Launch the plan's work on `stream`: directly, or, when the plan replays
// graphs (non-default streams only), through a HIP graph captured on the
// first call with a given (params, out, bound, stream) binding.
extern "C++" {
template <class Launch>
static sg_status graph_or_direct(sg_plan* p, const double* params_dev, double* out_dev, double* bound_dev,
                                 void* stream, Launch launch)
{
    if (!stream || !p->use_graph || !graphs_enabled()) return launch(stream);
    for (GraphEntry& g : p->graphs) {
        if (g.params == params_dev && g.out == out_dev && g.bound == bound_dev && g.stream == stream) {
            hipError_t e = hipGraphLaunch(g.exec, (hipStream_t)stream);
            if (e != hipSuccess) return hip_fail(p->ctx, e, "hipGraphLaunch");
            return SG_OK;
        }
    }
    // first call with this binding: capture the launches into a graph
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return fail(p->ctx, SG_ERR_CAPTURE, std::string("begin capture: ") + hipGetErrorString(e));
    const sg_status st = launch(stream);
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(s, &graph);
    if (st != SG_OK || e != hipSuccess || !graph) {
        if (graph) (void)hipGraphDestroy(graph);
        if (st != SG_OK) return st;
        return fail(p->ctx, SG_ERR_CAPTURE, std::string("capture: ") + hipGetErrorString(e));
    }
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(graph);
        return fail(p->ctx, SG_ERR_CAPTURE, std::string("instantiate: ") + hipGetErrorString(e));
    }
    if (p->graphs.size() >= 8) {   // keep the cache small
        (void)hipGraphExecDestroy(p->graphs.front().exec);
        (void)hipGraphDestroy(p->graphs.front().graph);
        p->graphs.erase(p->graphs.begin());
    }
    p->graphs.push_back(GraphEntry{params_dev, out_dev, bound_dev, stream, graph, exec});
    e = hipGraphLaunch(exec, s);
    if (e != hipSuccess) return hip_fail(p->ctx, e, "hipGraphLaunch");
    return SG_OK;
}
}  // extern "C++"

sg_status sg_plan_execute(sg_plan* p, const double* params_dev, double* out_dev, double* bound_dev, void* stream)
{
    if (!p) return SG_ERR_INVALID_ARGUMENT;
    if (!params_dev || !out_dev) return fail(p->ctx, SG_ERR_INVALID_ARGUMENT, "NULL params or out");
    if (p->blocked) return blocked_execute(p, params_dev, out_dev, bound_dev, stream);
    return graph_or_direct(p, params_dev, out_dev, bound_dev, stream,
                           [&](void* st) { return plan_launch(p, params_dev, out_dev, bound_dev, st); });
}

// The block variant's three launches (gather, forward over the blocks,
// combine), as one graph when the plan replays graphs.
static sg_status blocked_execute(sg_plan* p, const double* params_dev, double* out_dev, double* bound_dev,
                                 void* stream)
{
    BlockedPart& B = *p->blocked;
    return graph_or_direct(p, params_dev, out_dev, bound_dev, stream, [&](void* st) {
        int rc = launch_block_gather(B.d_subs, B.nsub, B.m, params_dev, B.d_params, B.d_phase, st);
        if (rc != 0) return hip_fail(p->ctx, (hipError_t)rc, "block gather launch");
        sg_status s2 = plan_launch(B.inner, B.d_params, B.d_out, B.d_bound, st);
        if (s2 != SG_OK) return s2;
        rc = launch_block_combine(B.d_bprobs, p->n, B.d_out, B.d_bound, B.d_phase, params_dev, out_dev, bound_dev, st);
        if (rc != 0) return hip_fail(p->ctx, (hipError_t)rc, "block combine launch");
        return SG_OK;
    });
}

sg_status sg_plan_create_blocked(sg_context* ctx, const sg_problem* problems, int32_t n, int32_t precision,
                                 int32_t block_dims, sg_plan** plan)
{
    if (!ctx || !plan) return SG_ERR_INVALID_ARGUMENT;
    *plan = nullptr;
    if (!problems || n < 1) return fail(ctx, SG_ERR_INVALID_ARGUMENT, "empty problem list");
    if (block_dims < 1) return fail(ctx, SG_ERR_INVALID_ARGUMENT, "block_dims must be >= 1");
    for (int i = 0; i < n; ++i) {
        sg_status st = validate_problem(ctx, problems[i], i);
        if (st != SG_OK) return st;
    }
    // block sub-problems in integrand order, blocks in coordinate order
    // (oscillatory quadratic families: real part, then imaginary part;
    // oscillatory: one sub-problem per block, its phase cancelled, rotated
    // back by the combine); their parameters are laid out contiguously in
    // the plan's block array
    std::vector<sg_problem> sub;
    std::vector<BlockSub> gs;
    std::vector<BlockProb> bp(n);
    int64_t off = 0;
    uint64_t eff = 0;
    for (int i = 0; i < n; ++i) {
        const sg_problem& P = problems[i];
        const int K = P.q - P.d;
        const int nb = (P.d + block_dims - 1) / block_dims;
        // parts per block: two sweeps for the complex-sweep families (their
        // block sums are complex), one phase-cancelled sweep for the linear
        // oscillatory family (its sum is real, the phase a rotation)
        const bool two_parts = family_complex(P.family);
        const int part_lo = two_parts ? 1 : P.family == SG_FAMILY_OSCILLATORY ? 3 : 0;
        const int part_hi = two_parts ? 2 : part_lo;
        if (sub.size() + (size_t)nb * (two_parts ? 2 : 1) > (size_t)INT32_MAX)
            return fail(ctx, SG_ERR_UNSUPPORTED, "too many blocks");
        bp[i].param_offset = P.param_offset;
        bp[i].first_sub = (int32_t)sub.size();
        bp[i].nblocks = nb;
        bp[i].family = P.family;
        bp[i].out_index = i;
        bp[i].d = P.d;
        bp[i].block_dims = block_dims;
        uint64_t pts = 1;
        for (int b = 0; b < nb; ++b) {
            const int start = b * block_dims, len = std::min(block_dims, P.d - start);
            uint64_t nrep = 0;
            sg_status st = counts(len, len + K, P.rule, nullptr, &nrep, nullptr);
            pts = sat_mul(pts, st == SG_OK ? nrep : UINT64_MAX);
            for (int part = part_lo; part <= part_hi; ++part) {
                BlockSub g{};
                g.src_off = P.param_offset;
                g.dst_off = off;
                g.start = start;
                g.len = len;
                g.d = P.d;
                g.family = P.family;
                g.part = part;
                gs.push_back(g);
                sub.push_back(sg_problem{len, len + K, P.rule, P.family, off});
                off += P.family == SG_FAMILY_OSCILLATORY ? 1 + (int64_t)len
                       : P.family == SG_FAMILY_OSCILLATORY_QUADRATIC ? 1 + 2 * (int64_t)len
                       : P.family == SG_FAMILY_OSCILLATORY_QUADRATIC_LINEAR ? 1 + 3 * (int64_t)len
                       : (P.family == SG_FAMILY_PRODUCT_PEAK || P.family == SG_FAMILY_GAUSSIAN) ? 2 * (int64_t)len
                                                                                                : len;
            }
        }
        eff = sat_add(eff, pts);
    }
    sg_plan* inner = nullptr;
    sg_status st = sg_plan_create(ctx, sub.data(), (int32_t)sub.size(), precision, &inner);
    if (st != SG_OK) return st;
    PlanOwner p(new sg_plan());
    p->ctx = ctx;
    p->precision = precision;
    p->n = n;
    p->problems.assign(problems, problems + n);
    p->blocked = new BlockedPart();
    BlockedPart& B = *p->blocked;
    B.m = block_dims;
    B.inner = inner;
    B.nsub = (int)sub.size();
    p->info = inner->info;
    p->info.effective_points = eff;
    p->info.fp64_complex = 0;
    for (int i = 0; i < n; ++i)
        if (family_complex(problems[i].family)) p->info.fp64_complex++;
    inner->use_graph = false;      // graphs, when chosen, hold all three launches
    inner->info.graph = 0;
    p->use_graph = false;
    p->info.graph = 0;
    ctx->live_plans++;
    if ((st = upload(ctx, &B.d_subs, gs.data(), gs.size())) != SG_OK) { sg_plan_destroy(p.release()); return st; }
    if ((st = upload(ctx, &B.d_bprobs, bp.data(), bp.size())) != SG_OK) { sg_plan_destroy(p.release()); return st; }
    hipError_t e = hipMalloc((void**)&B.d_params, std::max<int64_t>(1, off) * sizeof(double));
    if (e == hipSuccess) e = hipMalloc((void**)&B.d_out, (size_t)B.nsub * sizeof(double));
    if (e == hipSuccess) e = hipMalloc((void**)&B.d_bound, (size_t)B.nsub * sizeof(double));
    if (e == hipSuccess) e = hipMalloc((void**)&B.d_phase, 2 * (size_t)B.nsub * sizeof(double));
    if (e != hipSuccess) {
        sg_plan_destroy(p.release());
        return fail(ctx, SG_ERR_OUT_OF_MEMORY, std::string("hipMalloc: ") + hipGetErrorString(e));
    }
    *plan = p.release();
    return SG_OK;
}

sg_status sg_plan_execute_grad(sg_plan* p, const double* params_dev, const double* grad_out_dev,
                               double* grad_params_dev, void* stream)
{
    if (!p) return SG_ERR_INVALID_ARGUMENT;
    if (!params_dev || !grad_out_dev || !grad_params_dev)
        return fail(p->ctx, SG_ERR_INVALID_ARGUMENT, "NULL params, grad_out or grad_params");
    if (p->blocked) return fail(p->ctx, SG_ERR_UNSUPPORTED, "the block variant has no reverse sweep");
    if (!p->params_disjoint)
        return fail(p->ctx, SG_ERR_INVALID_ARGUMENT,
                    "problems share parameters: the reverse sweep needs disjoint parameter ranges");
    if (!p->d_ws) {
        hipError_t e = hipMalloc((void**)&p->d_ws, std::max<size_t>(1, p->ws_elems) * sizeof(double));
        if (e != hipSuccess) {
            p->d_ws = nullptr;
            return fail(p->ctx, SG_ERR_OUT_OF_MEMORY, std::string("workspace: ") + hipGetErrorString(e));
        }
    }
    const int rc = launch_adjoint(p->precision, p->kmax == kKmaxGauss, p->nwg, p->d_wgs, p->d_probs, p->d_pool64,
                                  p->d_pool32, params_dev, grad_out_dev, grad_params_dev, p->d_ws, stream);
    if (rc != 0) return hip_fail(p->ctx, (hipError_t)rc, "adjoint launch");
    if (p->noscq) {
        const int rq = launch_oscq_grad(p->noscq, p->d_oscq, p->d_pool64, params_dev, grad_out_dev, grad_params_dev,
                                        p->d_ws, stream);
        if (rq != 0) return hip_fail(p->ctx, (hipError_t)rq, "oscillatory-quadratic reverse sweep launch");
    }
    return SG_OK;
}

sg_status sg_plan_get_info(const sg_plan* p, sg_plan_info* info)
{
    if (!p || !info) return SG_ERR_INVALID_ARGUMENT;
    *info = p->info;
    return SG_OK;
}

// After the inner plan's schedule changed: the outer plan keeps the graph
// choice (its graphs hold the inner launch, so they are rebuilt).
static void blocked_sync_info(sg_plan* p, bool graph)
{
    sg_plan* in = p->blocked->inner;
    in->use_graph = false;
    in->info.graph = 0;
    destroy_graphs(in);
    destroy_graphs(p);
    p->use_graph = graph;
    p->info.graph = graph ? 1 : 0;
    p->info.grid_blocks = in->info.grid_blocks;
    p->info.coords_per_lane = in->info.coords_per_lane;
    p->info.max_group = in->info.max_group;
    p->info.persistent = in->info.persistent;
    p->info.cost_scaled = in->info.cost_scaled;
    p->info.balanced = in->info.balanced;
}

sg_status sg_plan_autotune(sg_plan* p, const double* params_dev, double* out_dev, void* stream)
{
    if (!p || !params_dev || !out_dev) return SG_ERR_INVALID_ARGUMENT;
    if (p->blocked) {
        BlockedPart& B = *p->blocked;
        const int rc = launch_block_gather(B.d_subs, B.nsub, B.m, params_dev, B.d_params, B.d_phase, stream);
        if (rc != 0) return hip_fail(p->ctx, (hipError_t)rc, "block gather launch");
        sg_status st = sg_plan_autotune(B.inner, B.d_params, B.d_out, stream);
        blocked_sync_info(p, false);
        if (st != SG_OK || !stream) return st;
        // direct launches or one graph of the three: keep the faster
        hipEvent_t e0, e1;
        if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
            return fail(p->ctx, SG_ERR_DEVICE, "hipEventCreate");
        float ms[2] = {0.f, 0.f};
        for (int g = 0; g < 2 && st == SG_OK; ++g) {
            p->use_graph = g == 1;
            if ((st = sg_plan_execute(p, params_dev, out_dev, nullptr, stream)) != SG_OK) break;   // warm / capture
            (void)hipEventRecord(e0, (hipStream_t)stream);
            for (int r = 0; r < 20; ++r) sg_plan_execute(p, params_dev, out_dev, nullptr, stream);
            (void)hipEventRecord(e1, (hipStream_t)stream);
            hipError_t e = hipEventSynchronize(e1);
            if (e != hipSuccess) { st = hip_fail(p->ctx, e, "autotune sync"); break; }
            (void)hipEventElapsedTime(&ms[g], e0, e1);
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        blocked_sync_info(p, st == SG_OK && ms[1] < ms[0]);
        return st;
    }
    hipStream_t s = (hipStream_t)stream;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return fail(p->ctx, SG_ERR_DEVICE, "hipEventCreate");
    const FwdSched saved = p->sched;
    const bool saved_g = p->use_graph;
    FwdSched best = saved;
    bool best_g = saved_g;
    float best_ms = 1e30f;
    const int reps = 20;
    const int cpls[6] = {1, 2, 3, 4, 8, 16};
    const int gmaxs[3] = {1, 2, 4};
    sg_status st = SG_OK;
    // candidates: coordinates per lane (uniform or cost-scaled) x waves per
    // problem x (hardware dispatch | persistent work queue) x (graph replay |
    // direct launch); the graph variant is only timed on a non-default stream
    for (int c : cpls) {
        for (int gq = 0; gq < 12; ++gq) {
            const int gm = gmaxs[gq % 3];
            FwdSched sc;
            sc.balanced = 0;
            sc.cpl = c;
            sc.gmax = gm;
            sc.persistent = (gq / 3) % 2 == 1;
            sc.cost_scaled = gq >= 6;
            if ((st = plan_repack(p, sc)) != SG_OK) break;
            destroy_graphs(p);
            for (int g = 0; g < (stream ? 2 : 1); ++g) {
                p->use_graph = g == 1;
                if ((st = sg_plan_execute(p, params_dev, out_dev, nullptr, stream)) != SG_OK) break;   // warm / capture
                (void)hipEventRecord(e0, s);
                for (int r = 0; r < reps; ++r) sg_plan_execute(p, params_dev, out_dev, nullptr, stream);
                (void)hipEventRecord(e1, s);
                hipError_t e = hipEventSynchronize(e1);
                if (e != hipSuccess) { st = hip_fail(p->ctx, e, "autotune sync"); break; }
                float ms = 0.f;
                (void)hipEventElapsedTime(&ms, e0, e1);
                if (ms < best_ms) { best_ms = ms; best = sc; best_g = p->use_graph; }
            }
            if (st != SG_OK) break;
        }
        if (st != SG_OK) break;
    }
    // balanced schedules: 1..4 equal-cost waves per SIMD
    for (int m = 1; m <= 4 && st == SG_OK; ++m) {
        FwdSched sc;
        sc.balanced = m;
        if ((st = plan_repack(p, sc)) != SG_OK) break;
        destroy_graphs(p);
        for (int g = 0; g < (stream ? 2 : 1); ++g) {
            p->use_graph = g == 1;
            if ((st = sg_plan_execute(p, params_dev, out_dev, nullptr, stream)) != SG_OK) break;
            (void)hipEventRecord(e0, s);
            for (int r = 0; r < reps; ++r) sg_plan_execute(p, params_dev, out_dev, nullptr, stream);
            (void)hipEventRecord(e1, s);
            hipError_t e = hipEventSynchronize(e1);
            if (e != hipSuccess) { st = hip_fail(p->ctx, e, "autotune sync"); break; }
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, e0, e1);
            if (ms < best_ms) { best_ms = ms; best = sc; best_g = p->use_graph; }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    destroy_graphs(p);
    sg_status st2 = plan_repack(p, st == SG_OK ? best : saved);
    p->use_graph = st == SG_OK ? best_g : saved_g;
    if (st != SG_OK) return st;
    if (st2 != SG_OK) return st2;
    p->ctx->tuned[p->tune_key] = std::make_pair(best, best_g);
    p->info.graph = p->use_graph ? 1 : 0;
    return SG_OK;
}

sg_status sg_plan_set_schedule(sg_plan* p, int32_t coords_per_lane, int32_t max_group, int32_t cost_scaled,
                               int32_t persistent, int32_t graph)
{
    if (!p) return SG_ERR_INVALID_ARGUMENT;
    if (coords_per_lane < 1 || coords_per_lane > 64 || (max_group != 1 && max_group != 2 && max_group != 4) ||
        (cost_scaled != 0 && cost_scaled != 1) || (persistent != 0 && persistent != 1) || (graph != 0 && graph != 1))
        return fail(p->ctx, SG_ERR_INVALID_ARGUMENT, "schedule out of range");
    if (p->blocked) {
        sg_status st = sg_plan_set_schedule(p->blocked->inner, coords_per_lane, max_group, cost_scaled, persistent, 0);
        blocked_sync_info(p, graph == 1);
        return st;
    }
    FwdSched sc;
    sc.balanced = 0;
    sc.cpl = coords_per_lane;
    sc.gmax = max_group;
    sc.cost_scaled = cost_scaled == 1;
    sc.persistent = persistent == 1;
    destroy_graphs(p);
    sg_status st = plan_repack(p, sc);
    if (st != SG_OK) return st;
    p->use_graph = graph == 1;
    p->info.graph = graph;
    return SG_OK;
}

sg_status sg_plan_set_schedule_balanced(sg_plan* p, int32_t waves_per_simd, int32_t graph)
{
    if (!p) return SG_ERR_INVALID_ARGUMENT;
    if (waves_per_simd < 1 || waves_per_simd > 8 || (graph != 0 && graph != 1))
        return fail(p->ctx, SG_ERR_INVALID_ARGUMENT, "schedule out of range");
    if (p->blocked) {
        sg_status st = sg_plan_set_schedule_balanced(p->blocked->inner, waves_per_simd, 0);
        blocked_sync_info(p, graph == 1);
        return st;
    }
    FwdSched sc;
    sc.balanced = waves_per_simd;
    destroy_graphs(p);
    sg_status st = plan_repack(p, sc);
    if (st != SG_OK) return st;
    p->use_graph = graph == 1;
    p->info.graph = graph;
    return SG_OK;
}

sg_status sg_plan_destroy(sg_plan* p)
{
    if (!p) return SG_OK;
    if (p->ctx) p->ctx->live_plans--;
    plan_free(p);
    return SG_OK;
}

// Release a plan's device buffers, graphs, block part and the plan itself.
static void plan_free(sg_plan* p)
{
    if (p->blocked) {
        BlockedPart* B = p->blocked;
        sg_plan_destroy(B->inner);
        (void)hipFree(B->d_subs);
        (void)hipFree(B->d_bprobs);
        (void)hipFree(B->d_params);
        (void)hipFree(B->d_out);
        (void)hipFree(B->d_bound);
        (void)hipFree(B->d_phase);
        delete B;
        p->blocked = nullptr;
    }
    destroy_graphs(p);
    (void)hipFree(p->d_oscq);
    (void)hipFree(p->d_probs);
    (void)hipFree(p->d_wgs);
    (void)hipFree(p->d_fwd);
    (void)hipFree(p->d_queue);
    (void)hipFree(p->d_ws);
    (void)hipFree(p->d_pool64);
    (void)hipFree(p->d_pool32);
    delete p;
}

// Arguments of the plan-free path (sg_integrate, sg_integrate_noalloc).
static sg_status check_one(sg_context* ctx, const sg_problem* problem, int32_t precision, const double* params_dev,
                           const double* out_dev)
{
    if (!problem || !params_dev || !out_dev) return fail(ctx, SG_ERR_INVALID_ARGUMENT, "NULL argument");
    if (precision != SG_PREC_FP64 && precision != SG_PREC_FP32_COMPENSATED && precision != SG_PREC_FP32_FP64_SUM)
        return fail(ctx, SG_ERR_INVALID_ARGUMENT, "unknown precision");
    return validate_problem(ctx, *problem, 0);
}

sg_status sg_integrate(sg_context* ctx, const sg_problem* problem, int32_t precision, const double* params_dev,
                       double* out_dev, double* bound_dev, void* stream)
{
    if (!ctx) return SG_ERR_INVALID_ARGUMENT;
    sg_status st = check_one(ctx, problem, precision, params_dev, out_dev);
    if (st != SG_OK) return st;
    const int d = problem->d, K = problem->q - problem->d;
    const int G = one_workgroups(d, family_complex(problem->family));
    if (G > 1 && !ctx->one_ws) {
        // the split launches' scratch: allocated once per context, counter
        // zeroed once; every launch leaves it at zero
        const size_t words = (size_t)noalloc_capacity_words();
        hipError_t e = hipMalloc((void**)&ctx->one_ws, words * sizeof(double));
        if (e != hipSuccess) {
            ctx->one_ws = nullptr;
            return fail(ctx, SG_ERR_OUT_OF_MEMORY, std::string("hipMalloc: ") + hipGetErrorString(e));
        }
        e = hipMemset(ctx->one_ws, 0, words * sizeof(double));
        if (e != hipSuccess) {
            (void)hipFree(ctx->one_ws);
            ctx->one_ws = nullptr;
            return hip_fail(ctx, e, "hipMemset");
        }
    }
    const int rc = family_complex(problem->family)
                       ? launch_oscq(precision, d, K, problem->rule, G,
                                     problem->family == SG_FAMILY_OSCILLATORY_QUADRATIC_LINEAR ? 1 : 0, nullptr,
                                     nullptr, params_dev, out_dev, bound_dev, ctx->one_ws, stream)
                       : launch_one(precision, d, K, problem->rule, problem->family, G, params_dev, out_dev,
                                    bound_dev, ctx->one_ws, stream);
    if (rc != 0) return hip_fail(ctx, (hipError_t)rc, "plan-free launch");
    return SG_OK;
}

sg_status sg_integrate_noalloc(sg_context* ctx, const sg_problem* problem, int32_t precision,
                               const double* params_dev, double* out_dev, double* bound_dev, void* stream)
{
    if (!ctx) return SG_ERR_INVALID_ARGUMENT;
    sg_status st = check_one(ctx, problem, precision, params_dev, out_dev);
    if (st != SG_OK) return st;
    if (!ctx->noalloc) return fail(ctx, SG_ERR_DEVICE, "no scratch array on this device");
    const int rc = noalloc_launch(ctx->noalloc, precision, problem->d, problem->q - problem->d, problem->rule,
                                  problem->family, params_dev, out_dev, bound_dev, stream);
    if (rc == -1) return fail(ctx, SG_ERR_UNSUPPORTED, "problem needs more scratch than the fixed array holds");
    if (rc != 0) return hip_fail(ctx, (hipError_t)rc, "allocation-free launch");
    return SG_OK;
}

}  // extern "C"

const char* sg_version(void) { return SG_VERSION_STRING; }

sg_status sg_context_save_tuning(const sg_context* ctx, const char* path)
{
    if (!ctx || !path) return SG_ERR_INVALID_ARGUMENT;
    sg_context* c = const_cast<sg_context*>(ctx);
    TuneFile f;
    f.version = SG_VERSION_STRING;
    f.arch = ctx->arch;
    f.compute_units = ctx->n_cu;
    for (const auto& kv : ctx->tuned) {
        TuneRecord r;
        r.key = kv.first;
        const FwdSched& sc = kv.second.first;
        r.cpl = sc.cpl;
        r.gmax = sc.gmax;
        r.cost_scaled = sc.cost_scaled ? 1 : 0;
        r.persistent = sc.persistent ? 1 : 0;
        r.balanced = sc.balanced;
        r.graph = kv.second.second ? 1 : 0;
        f.entries.push_back(r);
    }
    const std::string text = tune_file_write(f);
    const std::string tmp = std::string(path) + ".tmp";
    FILE* fp = std::fopen(tmp.c_str(), "wb");
    if (!fp) return fail(c, SG_ERR_INVALID_ARGUMENT, std::string("cannot write ") + tmp);
    const bool ok = std::fwrite(text.data(), 1, text.size(), fp) == text.size();
    if (std::fclose(fp) != 0 || !ok) {
        std::remove(tmp.c_str());
        return fail(c, SG_ERR_INVALID_ARGUMENT, std::string("cannot write ") + tmp);
    }
    if (std::rename(tmp.c_str(), path) != 0) {
        std::remove(tmp.c_str());
        return fail(c, SG_ERR_INVALID_ARGUMENT, std::string("cannot replace ") + path);
    }
    return SG_OK;
}

sg_status sg_context_load_tuning(sg_context* ctx, const char* path, int32_t* n_loaded)
{
    if (!ctx || !path) return SG_ERR_INVALID_ARGUMENT;
    if (n_loaded) *n_loaded = 0;
    FILE* fp = std::fopen(path, "rb");
    if (!fp) return fail(ctx, SG_ERR_INVALID_ARGUMENT, std::string("cannot open ") + path);
    std::string text;
    char buf[4096];
    size_t got = 0;
    while ((got = std::fread(buf, 1, sizeof buf, fp)) > 0) {
        text.append(buf, got);
        if (text.size() > ((size_t)1 << 24)) {
            std::fclose(fp);
            return fail(ctx, SG_ERR_INVALID_ARGUMENT, "autotune file larger than 16 MiB");
        }
    }
    std::fclose(fp);
    TuneFile f;
    std::string err;
    if (!tune_file_read(text, f, err)) return fail(ctx, SG_ERR_INVALID_ARGUMENT, "autotune file: " + err);
    // results of another build or device do not apply: load nothing
    if (f.version != SG_VERSION_STRING || f.arch != ctx->arch || f.compute_units != ctx->n_cu) return SG_OK;
    for (const TuneRecord& r : f.entries) {
        FwdSched sc;
        sc.cpl = r.cpl;
        sc.gmax = r.gmax;
        sc.cost_scaled = r.cost_scaled == 1;
        sc.persistent = r.persistent == 1;
        sc.balanced = r.balanced;
        ctx->tuned[r.key] = std::make_pair(sc, r.graph == 1);
    }
    if (n_loaded) *n_loaded = (int32_t)f.entries.size();
    return SG_OK;
}
