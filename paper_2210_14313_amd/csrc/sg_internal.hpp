// Internal declarations shared by the host runtime and the kernel launchers.
// Not part of the ABI (see include/sgmdi.h).
#pragma once

#include <cstdint>
#include <map>
#include <memory>
#include <string>
#include <tuple>
#include <vector>

#include "sgmdi.h"

namespace sg {

constexpr int kMaxK = SG_MAX_K;
// Launch class of forward plans holding gaussian problems (kernels built
// for K <= kMaxK with that family).
constexpr int kKmaxGauss = kMaxK + 1;

// ---------------------------------------------------------------- 1-D rules
// Number of nodes of the level-l rule (Section 2.2); -1 if unknown/too big.
long rule_npoints(int rule, int level);
bool rule_is_known(int rule);
bool rule_is_nested(int rule);
// Level-l nodes/weights on [0,1], ascending, computed in long double.
bool rule_nodes(int rule, int level, std::vector<long double>& x, std::vector<long double>& w);

// Hierarchical (difference-rule) table for one (rule, K).
//
// The Smolyak sum over the window equals the sum over all l with excess
// |l| - d <= K of the tensor products of difference rules
// Delta^1 = J^1, Delta^{e+1} = J^{e+1} - J^e (the reading of (2.9) as a
// summation by coordinates).  Every difference rule with e >= 1 has weights
// summing to 0 and is symmetric about 1/2, so it only sees the even part of
// a centred factor g(1/2 + y)/g(1/2) - 1.  The table therefore lists node
// PAIRS {1/2 - y, 1/2 + y}, y > 0, and for each pair and each e >= 1 the
// weight dW[e][p] the pair's nodes carry in Delta^{e+1}.
//
// Pairs are grouped by the level L at which they first enter; pair p of
// level L carries non-zero weights for
//   nested rules (trapezoid, Clenshaw-Curtis):  e = L-1 .. K
//   Gauss-Legendre (levels share only 1/2):     e = L-1 and e = L (if <= K).
struct DeltaTable {
    int rule = 0, K = 0, npairs = 0;
    bool nested = true;
    std::vector<int> level_begin;          // size K+3; pairs of level L: [lb[L], lb[L+1])
    std::vector<double> y;                 // npairs, y_p > 0
    std::vector<double> dw;                // (K+1) x npairs, row 0 unused (zero)
    std::vector<float> y32, dw_hi, dw_lo;  // FP32 copies; dw = dw_hi + dw_lo to ~2^-48
    std::vector<double> wabs;              // npairs: sum_e |dW[e][p]| (error bound)
};
bool build_delta_table(int rule, int K, DeltaTable& t, std::string& err);

// ------------------------------------------------------------ integer layer
// Exact unsigned binomial with overflow report (result >= 2^64 -> false).
bool binom_u64(uint64_t n, uint64_t k, uint64_t& out);
sg_status counts(int d, int q, int rule, uint64_t* n_multi, uint64_t* n_rep, uint64_t* n_unique);
sg_status unrank(int d, int q, uint64_t rank, int32_t* coords, int32_t* levels, int32_t* nnz);

// ------------------------------------------------------- static rule layout
// Structure classes of the difference-rule tables, fixed per (class, K):
// pairs entering at level L and the e-range [elo, ehi] their nodes carry
// weights in.  The kernels unroll over this structure at compile time; the
// host writes the tables in exactly this order (and checks the counts).
// RC_GP: Gauss-Patterson with the level map 1, 3, 3, 7, 7, 7, 15, ...: new
// pairs enter at levels 2 (1), 4 (2) and 7 (4); the repeated levels give
// difference rules that vanish (their rows hold zero weights).
enum { RC_NESTED = 0, RC_GL2 = 1, RC_GLP = 2, RC_GP = 3 };

constexpr int rule_class_of(int rule)
{
    return (rule == SG_RULE_TRAPEZOID || rule == SG_RULE_CLENSHAW_CURTIS) ? RC_NESTED
           : rule == SG_RULE_GAUSS_PATTERSON ? RC_GP
           : rule == SG_RULE_GAUSS_LEGENDRE ? RC_GL2 : RC_GLP;
}
constexpr int rc_pairs(int rc, int L)
{
    return L < 2 ? 0
           : rc == RC_NESTED ? (L == 2 ? 1 : (1 << (L - 3)))
           : rc == RC_GP ? (L == 2 ? 1 : L == 4 ? 2 : L == 7 ? 4 : 0)
           : rc == RC_GL2 ? L - 1 : L / 2;
}
constexpr int rc_elo(int L) { return L - 1; }
constexpr int rc_ehi(int rc, int K, int L) { return (rc == RC_NESTED || rc == RC_GP) ? K : (L < K ? L : K); }
// FP64 record of one pair: y, dW[elo..ehi], sum_e |dW|
constexpr int rc_rec64(int rc, int K, int L) { return rc_ehi(rc, K, L) - rc_elo(L) + 3; }
// FP32 record of one pair: (dW_hi, dW_lo) for e = elo..ehi
constexpr int rc_rec32(int rc, int K, int L) { return 2 * (rc_ehi(rc, K, L) - rc_elo(L) + 1); }
constexpr int rc_off64(int rc, int K, int L)
{
    int o = 0;
    for (int l = 2; l < L; ++l) o += rc_pairs(rc, l) * rc_rec64(rc, K, l);
    return o;
}
constexpr int rc_off32(int rc, int K, int L)
{
    int o = 0;
    for (int l = 2; l < L; ++l) o += rc_pairs(rc, l) * rc_rec32(rc, K, l);
    return o;
}

// ------------------------------------------------------------------- device
// Per-problem record in device memory (plan order = longest first).
struct ProbDev {
    int32_t d, K, family, rule;    // rule: sg_rule (the structure class follows from it)
    int64_t param_offset;
    int64_t off64;                 // record table in pool64
    int64_t off32;                 // record table in pool32
    int32_t out_index;             // position in the caller's problem order
    int32_t waves;                 // waves this problem spans inside its workgroup (1, 2 or 4)
    int64_t ws_off;                // reverse sweep: this problem's d*K slots in the workspace
};

// One workgroup = 4 waves; wave w works on problem slot[w].prob (or idles
// when prob < 0) as wave `rank` of a group of `group` waves.
struct WaveSlot {
    ProbDev p;         // copy of the problem record (saves a dependent load)
    int32_t prob;      // plan index of the problem, -1 for an idle wave
    int16_t rank, group;
};
struct WGDesc {
    WaveSlot slot[4];
};

// ----------------------------------------------------- forward schedule
// One problem as a forward lane segment sees it.
struct FwdSeg {
    int32_t d;
    int32_t out_index;             // position in the caller's problem order
    int64_t param_offset;
};

// One wave of the forward sweep.  All its problems share one class
// (K, rule, family), so the wave runs one code path.  Either up to
// kWaveProbs problems sit side by side on 2^lw lanes each (group == 1), or
// one problem spans `group` waves of 64 lanes (lw == 6) of one workgroup and
// is merged through LDS.  A lane reads its segment record directly (one
// load, no index indirection).
constexpr int kWaveProbs = 16;
struct FwdWave {
    int16_t K, rule, family, lw;   // class; lw = log2(lanes per problem), 2..6
    int16_t rank, group;           // wave rank inside its group; group size (1, 2, 4)
    int16_t nprob;                 // problems in this wave (0: idle wave)
    int16_t grouped;               // in w[0] only: 1 if any wave of the workgroup has group > 1
    int32_t off64, off32;          // the class's record table in the pools
    int32_t pad2[2];
    FwdSeg seg[kWaveProbs];        // the problems, by lane segment
};
struct FwdWG {
    FwdWave w[4];
};

struct LaunchCfg {
    int block = 256;   // threads per workgroup (always 4 waves)
};

// Kernel launchers (sg_unrank.hip dispatches to sg_fwd*.hip / sg_adj*.hip).
// kmax: the largest K of the launched problems (selects the instantiation).
// queue == nullptr: one workgroup per descriptor; else the persistent
// work-queue kernel on qgrid workgroups (queue: two zeroed counters).
int launch_forward(int precision, int kmax, int nwg, const FwdWG* wgs, unsigned int* queue, int qgrid,
                   const double* pool64, const float* pool32, const double* params, double* out,
                   double* bound, void* stream);
// Resident workgroups of the persistent forward kernel on the current device.
int forward_capacity(int precision, int kmax);
// Reverse sweep; gauss: the plan holds gaussian problems (launches the
// instantiation built with that family).
int launch_adjoint(int precision, bool gauss, int nwg, const WGDesc* wgs, const ProbDev* probs,
                   const double* pool64, const float* pool32, const double* params, const double* gout,
                   double* grad, double* ws, void* stream);
int launch_unrank(int d, int q, uint64_t rank0, uint64_t count, int max_nnz,
                  const uint64_t* binom_table, int binom_rows, int32_t* coords, int32_t* levels,
                  int32_t* nnz, void* stream);
const char* device_error_string(int code);

// One integrand of the sweep split over G workgroups (sg_one.hpp): G
// workgroups of 256 threads, precision mode `precision`; scratch (G > 1):
// kOneHead + G * kOneWords doubles, the first 32-bit word (the arrival
// counter) zero before the launch and zero after it.
constexpr int kOneHead = 32;
constexpr int kOneWords = kMaxK + 4;
constexpr int kOneMaxG = 1024;   // workgroups of one split launch at most
int launch_one(int precision, int d, int K, int rule, int family, int G, const double* params, double* out,
               double* bound, double* scratch, void* stream);
// Workgroups for an integrand of d coordinates.  One workgroup, its threads
// holding several coordinates each, up to kOneSingle coordinates (the
// sweep's families) or kOneSingleComplex (the complex sweep, whose
// coordinates cost more): below those sizes the longer chains cost less
// than the cross-workgroup join (measured: d = 1000 in 3.8-4.5 us on one
// workgroup against 5.6-6.0 us on four).  Above them one coordinate per
// lane (256 per workgroup), at most kOneMaxG workgroups.
constexpr int kOneSingle = 2048;
constexpr int kOneSingleComplex = 512;
inline int one_workgroups(int d, bool complex_sweep)
{
    if (d <= (complex_sweep ? kOneSingleComplex : kOneSingle)) return 1;
    const int g = (d + 255) / 256;
    return g > kOneMaxG ? kOneMaxG : g;
}

// Allocation-free path (sg_noalloc.hip): the current device's fixed scratch
// array (0 or a HIP error code), a split launch on it (0, a HIP error code,
// or -1 if it would need more scratch than the array holds), and the array's
// size in doubles (also the size of a context's split-launch scratch).
int noalloc_scratch(double** ptr);
int noalloc_launch(double* ptr, int precision, int d, int K, int rule, int family, const double* params,
                   double* out, double* bound, void* stream);
long noalloc_capacity_words();

// Literal point-by-point path (sg_points.hip).
struct PointsLaunch {
    int d, K, e0, grid;
    uint64_t n_multi;
    const uint64_t* W;             // weak-composition counts, (K+1) rows of d+1 (device)
    const double* node_y;          // nodes - 1/2 of levels 1..K+1, concatenated (device)
    const double* node_w;          // their weights (device)
    int level_off[kMaxK + 3];      // level l occupies [level_off[l], level_off[l+1])
    double coef[kMaxK + 1];        // combination coefficient by excess
    int emax;                      // largest sum of n_l over the active coordinates of a multi-index
    int cmax;                      // largest size of its two combined frontiers (points_frontier_sizes)
    const double* params;          // the integrand's parameters (device)
    double* partial;               // 3 * 4 * grid doubles of workspace (device)
    double* out;                   // one double (device-accessible)
    double* bound;                 // NULL or one double (device-accessible)
};
int launch_points(int family, const PointsLaunch& L, void* stream);

// Frontier capacities of the point path for a rule whose level l has n[l]
// nodes (l = 1..K+1): over every ordered list of active levels (>= 2) with
// sum(l - 1) <= K, the largest sum of n_l (*emax) and the largest
// min over splits s of prod_{m<s} n + prod_{m>=s} n (*cmax).
void points_frontier_sizes(const int* n, int K, int* emax, int* cmax);

// Block (tensor-product) variant: one record per block sub-problem (gather)
// and one per integrand (ordered combine).
struct BlockSub {
    int64_t src_off;   // integrand's parameter offset in the caller's array
    int64_t dst_off;   // block's parameter offset in the plan's block array
    int32_t start;     // first coordinate of the block
    int32_t len;       // coordinates in the block
    int32_t d;         // integrand's dimension (product-peak: offset of u)
    int32_t family;
    int32_t part;      // 0: plain copy; oscillatory quadratic families: 1 = real part (w = 0),
                       // 2 = imaginary part (w = -1/4); oscillatory: 3 = the block's phase
                       // cancelled (w = -theta_b / 2 pi, theta_b = sum of a_t / 2 over the block)
    int32_t pad;
};
struct BlockProb {
    int64_t param_offset;   // integrand's parameter offset (oscillatory: w)
    int32_t first_sub;      // its first block sub-problem (oscillatory quadratic: two per block)
    int32_t nblocks;
    int32_t family;
    int32_t out_index;
    int32_t d;              // integrand's dimension
    int32_t block_dims;     // coordinates per block (the last block may hold fewer)
};
// phase: two doubles per block sub-problem, written by the gather for
// oscillatory blocks (theta_b and sum |a_t| / 2) and read by the combine.
int launch_block_gather(const BlockSub* subs, int nsub, int block_dims, const double* params, double* sub_params,
                        double* phase, void* stream);
int launch_block_combine(const BlockProb* probs, int n, const double* sub_out, const double* sub_bound,
                         const double* phase, const double* params, double* out, double* bound, void* stream);

// Record tables (FP64 and FP32 pools) of one (rule, K) in the static layout.
bool build_records(const DeltaTable& t, std::vector<double>& rec64, std::vector<float>& rec32,
                   std::string& err);

// Autotune results on disk (sg_context_save_tuning / _load_tuning): one
// record per tuned plan shape.
constexpr const char* kTuneFormat = "sgmdi-autotune-1";
struct TuneRecord {
    std::string key;   // plan shape: precision, count and a hash of the sorted (d, K, rule, family) list
    int cpl = 4, gmax = 4, cost_scaled = 0, persistent = 0, balanced = 0, graph = 0;
};
struct TuneFile {
    std::string version;    // SG_VERSION_STRING of the writer
    std::string arch;       // the device's architecture name
    int compute_units = 0;
    std::vector<TuneRecord> entries;
};
std::string tune_file_write(const TuneFile& f);
// Parse a document written by tune_file_write; false (with err) if it is
// malformed or any record is out of range.
bool tune_file_read(const std::string& text, TuneFile& f, std::string& err);

}  // namespace sg
