/*
 * sgmdi.h -- C ABI of the MI355X (gfx950) Smolyak sparse-grid quadrature
 * library (libsgmdi.so).
 *
 * The library evaluates the Smolyak rule of Section 2.1, equation (2.6),
 *
 *   Q_d^q(f) = sum_{q-d+1 <= |l| <= q} (-1)^(q-|l|) C(d-1, q-|l|)
 *              sum_{|l| fixed} (J^{l_1} x ... x J^{l_d}) f,
 *
 * with tensor sub-rules (2.7) built from the 1-D rules of Section 2.2, by a
 * dimension sweep in the spirit of the multilevel dimension iteration of
 * Section 3 (Algorithms 3.1-3.3, (3.9)-(3.11)): the coordinates are swept
 * and only clustered partial quantities per coordinate are carried, never
 * points.  For the supported integrand families every partial function of
 * (3.11) is a truncated polynomial in the remaining level budget (the gamma
 * recursion under (2.9)) times an affine phase / log-amplitude sum.
 *
 * Domain: the unit cube [0,1]^d (the paper's [-1,1]^d of (2.1) is an affine
 * image; rescale parameters on the caller's side).  Level q and the excess
 * budget K = q - d are those of (2.6).  Level 1 of every rule is the single
 * midpoint 1/2 with weight 1.
 *
 * Conventions for every function:
 *   - the return value is an sg_status; nothing is thrown across the ABI;
 *   - arguments are validated on the host before anything is launched;
 *     a rejected call launches nothing and writes no output;
 *   - "device" pointers are HIP device allocations owned by the caller
 *     (e.g. torch tensors' data_ptr()); the library keeps no caller pointer
 *     beyond the call, except that a plan using graph replay caches one
 *     captured graph per (params, out, bound, stream) binding and replays
 *     it while the binding is unchanged;
 *   - "stream" is a hipStream_t passed as void* (NULL = default stream);
 *     device work is asynchronous on that stream;
 *   - one context per host thread; contexts and plans are not thread-safe.
 *
 * Developer hooks read from the environment (none changes a result):
 *   SGMDI_SCHED=c,g[,p[,s]]  sg_plan_create: force the forward schedule of
 *                            new plans (c coordinates per lane, g waves per
 *                            integrand, p persistent queue 0/1, s
 *                            cost-scaled 0/1), for profiling;
 *   SGMDI_NO_GRAPH=1         sg_plan_execute: never replay a graph.
 */
#ifndef SGMDI_H
#define SGMDI_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SG_OK = 0,
    SG_ERR_INVALID_ARGUMENT = 1, /* bad d, q, rule, family, size or NULL pointer */
    SG_ERR_UNSUPPORTED = 2,      /* valid but beyond what the library supports (e.g. K > SG_MAX_K) */
    SG_ERR_OVERFLOW = 3,         /* an exact count does not fit in 64 bits */
    SG_ERR_OUT_OF_MEMORY = 4,    /* host or device allocation failed */
    SG_ERR_DEVICE = 5,           /* a HIP call failed; see sg_last_error */
    SG_ERR_CAPTURE = 6           /* graph capture or instantiation failed */
} sg_status;

/* 1-D rules, numbered as the paper's parameter r (Section 3.1, Section 5). */
typedef enum {
    SG_RULE_TRAPEZOID = 1,           /* (2.10): n_1 = 1, n_l = 2^(l-1)+1, nested */
    SG_RULE_CLENSHAW_CURTIS = 2,     /* (2.11): n_1 = 1, n_l = 2^(l-1)+1, nested */
    SG_RULE_GAUSS_PATTERSON = 3,     /* (2.12): Patterson extensions, nested, with the level
                                        map of Section 5.4: levels 1..10 have 1, 3, 3, 7, 7, 7,
                                        15, 15, 15, 15 points (K <= 8 uses at most 15) */
    SG_RULE_GAUSS_LEGENDRE = 4,      /* Gauss-Legendre with n_l = 2l-1 points */
    SG_RULE_GAUSS_LEGENDRE_PAPER = 5 /* (2.13): Gauss-Legendre with n_l = l points */
} sg_rule;

/* Integrand families; parameters are float64, per integrand, contiguous:
 *   EXP_SUM       f(x) = exp(sum_i c_i x_i)                      params c[d]
 *   OSCILLATORY   f(x) = cos(2 pi w + sum_i a_i x_i)              params w, a[d]
 *   PRODUCT_PEAK  f(x) = prod_i 1/(b_i^-2 + (x_i - u_i)^2)        params b[d], u[d]
 *   CORNER_PEAK   f(x) = (1 + sum_i a_i x_i)^-(d+1), a_i >= 0     params a[d]
 *   GAUSSIAN      f(x) = exp(sum_i c_i (x_i - u_i)^2)             params c[d], u[d]
 *   OSCILLATORY_QUADRATIC
 *                 f(x) = cos(2 pi w + sum_i a_i (x_i - u_i)^2)    params w, a[d], u[d]
 *   OSCILLATORY_QUADRATIC_LINEAR
 *                 f(x) = cos(2 pi w + sum_i (a_i (x_i - u_i)^2 + c_i x_i))
 *                                                               params w, a[d], u[d], c[d]
 * (PRODUCT_PEAK is the integrand of (4.4)/(5.2) with free widths/centres;
 * EXP_SUM generalises (4.5)/(5.1); OSCILLATORY generalises Table 5.7's;
 * GAUSSIAN covers (4.3) and the exponentials of (4.1)/(4.2) (c of either
 * sign; forward and reverse sweeps and point path), OSCILLATORY_QUADRATIC
 * their sines, and OSCILLATORY_QUADRATIC_LINEAR the sine of (4.2) with its
 * linear term (a coordinate may be quadratic, linear, both or neither).
 * CORNER_PEAK is a ridge function that does not factor per coordinate: the
 * point-by-point path sg_integrate_points only.  The two
 * OSCILLATORY_QUADRATIC families factor with complex per-coordinate
 * surpluses: the point path, sg_integrate, and plans (a sweep with complex
 * truncated products, one workgroup per integrand beside the forward
 * kernel), block variant included, in every precision mode (the node values
 * and within-rule sums follow the mode; products, phase and read-out are
 * FP64), and their reverse sweep (FP64 in every mode, one workgroup per
 * integrand).
 * Plans reject CORNER_PEAK with UNSUPPORTED.) */
typedef enum {
    SG_FAMILY_EXP_SUM = 0,
    SG_FAMILY_OSCILLATORY = 1,
    SG_FAMILY_PRODUCT_PEAK = 2,
    SG_FAMILY_CORNER_PEAK = 3,
    SG_FAMILY_GAUSSIAN = 4,
    SG_FAMILY_OSCILLATORY_QUADRATIC = 5,
    SG_FAMILY_OSCILLATORY_QUADRATIC_LINEAR = 6
} sg_family;

/* Arithmetic of the per-coordinate work (node values and within-rule sums).
 * The sweep's truncated-polynomial products and the read-out are FP64 in
 * every mode.  Node values of integrands whose parameters leave the FP32
 * series range (|parameter| > 2) are formed in FP64 and rounded once in the
 * FP32 modes. */
typedef enum {
    SG_PREC_FP64 = 0,
    SG_PREC_FP32_COMPENSATED = 1, /* FP32 node values, FP32 hi+lo weights,
                                     two-sum compensated FP32 accumulation */
    SG_PREC_FP32_FP64_SUM = 2     /* FP32 node values, FP64 weights and
                                     FP64 accumulation (the reverse sweep of
                                     such a plan runs in mode 1) */
} sg_precision;

/* Version of this library (also the key under which autotune results are
 * saved: results of another version are not loaded). */
#define SG_VERSION_STRING "0.2.0"

/* Largest excess budget K = q - d the GPU path accepts. */
#define SG_MAX_K 8

/* One integrand of a batch.  param_offset indexes the batch's float64
 * parameter array (in elements); see sg_family for the layout. */
typedef struct {
    int32_t d;      /* dimension, >= 1 */
    int32_t q;      /* level of (2.6), q >= d */
    int32_t rule;   /* sg_rule */
    int32_t family; /* sg_family */
    int64_t param_offset;
} sg_problem;

typedef struct sg_context sg_context;
typedef struct sg_plan sg_plan;

/* ---------------------------------------------------------------- context */

/* Create a context on the current HIP device.  The context owns the rule
 * cache, the autotune results and its plans' device buffers.
 * Errors: INVALID_ARGUMENT (ctx NULL), DEVICE (no usable device). */
sg_status sg_context_create(sg_context **ctx);

/* Destroy a context (NULL is accepted).  Plans created from it must be
 * destroyed first. */
sg_status sg_context_destroy(sg_context *ctx);

/* Static text for a status code. */
const char *sg_status_string(sg_status s);

/* Detail of the last failure on this context (including HIP error text);
 * valid until the next call on the context.  Never NULL. */
const char *sg_last_error(const sg_context *ctx);

/* SG_VERSION_STRING of the loaded library. */
const char *sg_version(void);

/* Autotune results on disk.  A context keeps the schedule sg_plan_autotune
 * chose for every plan shape it tuned (shape: precision mode, problem count
 * and the multiset of (d, K, rule, family)); plans created later with the
 * same shape start from it.  sg_context_save_tuning writes them all to a
 * JSON file (written to path.tmp, then renamed over path): the library
 * version, the device's architecture name and compute-unit count, and one
 * record per shape.  sg_context_load_tuning reads such a file into the
 * context, replacing records of the same shape; a file written by another
 * library version, or for another architecture or compute-unit count, loads
 * nothing (*n_loaded = 0, SG_OK).  n_loaded may be NULL.  Plans that exist
 * already keep their schedule.
 * Errors: INVALID_ARGUMENT (NULL, unreadable or unwritable file, malformed
 * content or an out-of-range record: then nothing is loaded). */
sg_status sg_context_save_tuning(const sg_context *ctx, const char *path);
sg_status sg_context_load_tuning(sg_context *ctx, const char *path, int32_t *n_loaded);

/* ------------------------------------------------------- host, exact, sync */

/* Exact counts for (d, q, rule) (Section 2.1):
 *   n_multi         multi-indices in the window q-d+1 <= |l| <= q of (2.6);
 *   n_points_rep    n_d^q, the point count with repetition;
 *   n_points_unique distinct points of the sparse grid (the union (2.4)
 *                   over the window).
 * Any output pointer may be NULL.  Errors: INVALID_ARGUMENT (d < 1, q < d,
 * unknown rule), UNSUPPORTED (K > 60, or a level of the window whose rule
 * has more than 2^16+1 nodes), OVERFLOW (a count >= 2^64). */
sg_status sg_counts(int32_t d, int32_t q, int32_t rule,
                    uint64_t *n_multi, uint64_t *n_points_rep, uint64_t *n_points_unique);

/* Nodes and weights of the level-l 1-D rule on [0,1] (Section 2.2,
 * (2.10)-(2.13)), ascending.  x and w must hold at least n_l entries; pass
 * NULL for both to query n_l only.  Errors: INVALID_ARGUMENT (unknown rule,
 * level < 1), UNSUPPORTED (n_l > 2^16+1). */
sg_status sg_rule_table(int32_t rule, int32_t level, double *x, double *w, int32_t *n);

/* Signed combination coefficient (-1)^(q-|l|) C(d-1, q-|l|) of (2.6) for
 * multi-indices of excess e = |l| - d.  Returns 0 for e outside the window.
 * Errors: INVALID_ARGUMENT, OVERFLOW (|coefficient| >= 2^63). */
sg_status sg_coefficient(int32_t d, int32_t q, int32_t e, int64_t *coef);

/* Multi-index of a given rank in the canonical order of the window of
 * (2.6): by excess e = |l| - d ascending, then by (l_1, ..., l_d) in
 * decreasing lexicographic order.  Output is sparse: the *nnz coordinates
 * with l_i >= 2 (ascending, 0-based) and their levels; coords/levels must
 * hold K entries.  Errors: INVALID_ARGUMENT (rank >= n_multi or bad d, q),
 * OVERFLOW (the window is not countable in 64 bits). */
sg_status sg_unrank(int32_t d, int32_t q, uint64_t rank,
                    int32_t *coords, int32_t *levels, int32_t *nnz);

/* ---------------------------------------------------- device, asynchronous */

/* Unrank `count` consecutive ranks rank0, rank0+1, ... on the device, one
 * workgroup per block of ranks (same order and output as sg_unrank).
 * coords_dev/levels_dev: count x max_nnz int32 (row-major, unused slots
 * -1 / 0), nnz_dev: count int32.  max_nnz must be >= K.
 * Errors: INVALID_ARGUMENT (range beyond n_multi, NULL, max_nnz < K),
 * OVERFLOW, DEVICE. */
sg_status sg_unrank_device(sg_context *ctx, int32_t d, int32_t q, uint64_t rank0, uint64_t count,
                           int32_t max_nnz, int32_t *coords_dev, int32_t *levels_dev,
                           int32_t *nnz_dev, void *stream);

/* Build a plan for a batch of n problems (host array) in one precision:
 * validates every problem, builds (or reuses) the rule tables, orders the
 * work longest-first, picks tile/schedule parameters (from the context's
 * autotune results when present) and uploads the plan to the device.
 * OSCILLATORY_QUADRATIC(_LINEAR) problems run on the complex sweep in the plan's
 * precision mode, one workgroup each, launched after the forward kernel on
 * the same stream.
 * Errors: INVALID_ARGUMENT (n < 1, NULL, a bad problem), UNSUPPORTED
 * (K > SG_MAX_K, a CORNER_PEAK problem), OUT_OF_MEMORY, DEVICE. */
sg_status sg_plan_create(sg_context *ctx, const sg_problem *problems, int32_t n,
                         int32_t precision, sg_plan **plan);

/* Block (tensor-product) variant of the rule, Algorithm 3.3 with step
 * m = block_dims > 1 ((3.8)-(3.11)): the coordinates of every integrand are
 * cut into consecutive blocks of block_dims (the last block shorter when it
 * does not divide d), each block gets its own sparse grid of level
 * d_b + (q - d) (the integrand's excess budget), and the rule is the tensor
 * product of the block rules -- the reading under which the paper's errors
 * grow in proportion to d/m (Tables 4.7-4.9, 5.1-5.4).  block_dims >= d is
 * the plain rule.  The integrand must factor over the blocks (every family
 * but CORNER_PEAK; the oscillatory ones as the real and imaginary parts of
 * a product of complex block factors).  The returned plan is used like any other
 * (sg_plan_execute, _autotune, _set_schedule, _get_info, _destroy) with the
 * same parameter layout and outputs.  Execution is three launches (block
 * parameter gather, forward over the blocks, ordered combine), launched
 * directly, or -- when sg_plan_set_schedule's graph flag is set or the
 * autotuner found it faster, on non-default streams only -- captured into
 * one HIP graph per (params, out, bound, stream) binding and replayed.
 * bound_dev receives a bound on
 * |result - exact value of the block rule| propagated from the blocks'
 * bounds.  sg_plan_execute_grad is not available (UNSUPPORTED).
 * effective_points counts the tensor product's points (saturating).
 * Errors: INVALID_ARGUMENT (block_dims < 1, as sg_plan_create), UNSUPPORTED
 * (corner-peak, K > SG_MAX_K), OUT_OF_MEMORY, DEVICE. */
sg_status sg_plan_create_blocked(sg_context *ctx, const sg_problem *problems, int32_t n,
                                 int32_t precision, int32_t block_dims, sg_plan **plan);

/* Evaluate every integrand of the plan.  params_dev: the batch's float64
 * parameter array (device); out_dev: n float64 results in problem order
 * (device-accessible: device memory, or the device alias of pinned host
 * memory from hipHostGetDevicePointer, which lets the host read results
 * without a copy); bound_dev: NULL or n float64 a-priori bounds on
 * |result - exact Smolyak value| (device-accessible).  Launched directly by default; when the
 * autotuner found graph replay faster (non-default streams only), the launch
 * is captured into a HIP graph on the first call with a given
 * (params, out, bound, stream) and replayed after.
 * Errors: INVALID_ARGUMENT (NULL plan/params/out), DEVICE, CAPTURE. */
sg_status sg_plan_execute(sg_plan *plan, const double *params_dev, double *out_dev,
                          double *bound_dev, void *stream);

/* Gradient of every result with respect to every parameter (reverse sweep):
 * grad_params_dev[k] = grad_out_dev[i] * dQ_i/dparams[k] for the parameters
 * k of problem i, same layout as params.  Parameters not used by any problem
 * are left untouched.  OSCILLATORY_QUADRATIC(_LINEAR) problems take a complex reverse
 * sweep of their own (FP64 in every mode, one workgroup per integrand,
 * launched after the real one on the same stream).
 * Errors: INVALID_ARGUMENT (also: problems whose parameter ranges overlap),
 * DEVICE, UNSUPPORTED (a block-variant plan). */
sg_status sg_plan_execute_grad(sg_plan *plan, const double *params_dev, const double *grad_out_dev,
                               double *grad_params_dev, void *stream);

/* Plan facts for reporting (all exact counts of the algorithmic work of one
 * forward launch; u64 counts saturate at 2^64-1):
 *   effective_points  sum over problems of n_d^q (points with repetition);
 *   units             sum over problems of d ((integrand, coordinate) pairs);
 *   pair_evals        centred node-pair evaluations (one per symmetric pair
 *                     {1/2 - y, 1/2 + y} of the union node set, per unit);
 *   macs              within-rule multiply-adds (difference-rule weights
 *                     times pair values), summed over units;
 *   merge_flops       floating-point operations of the truncated-polynomial
 *                     products of the sweep (K(K-1)/2 multiply-adds and K
 *                     adds per unit, multiply-add counted as 2);
 *   block_threads, grid_blocks: the forward launch shape the plan uses;
 *   coords_per_lane, max_group, cost_scaled: the forward schedule.  Each
 *   wave runs one class (K, rule, family) of integrands; an integrand of d
 *   coordinates gets the fewest lanes (a power of two, 4..64) that keep
 *   every lane at <= c coordinates, several integrands sharing a wave, or,
 *   when d > 64 * c, 64 lanes on up to max_group (1, 2, 4) waves of one
 *   workgroup; c = coords_per_lane, or with cost_scaled = 1,
 *   floor(coords_per_lane * (largest per-coordinate cost of the plan) /
 *   (this class's per-coordinate cost)), capped at 64;
 *   graph: 1 if executions on a non-default stream replay a captured graph,
 *   0 if they launch directly;
 *   persistent: 1 if the forward launch is the persistent work-queue kernel
 *   (a grid of the device's resident capacity popping workgroup
 *   descriptors, longest first, from a per-plan queue that each launch
 *   leaves reset; executions of such a plan must not overlap in time), 0 if
 *   the hardware dispatches one workgroup per descriptor (the four knobs are
 *   chosen by sg_plan_autotune);
 *   balanced: 0, or the waves per SIMD of the balanced schedule
 *   (sg_plan_set_schedule_balanced), which replaces coords_per_lane,
 *   max_group and cost_scaled;
 *   fp64_complex: how many of the plan's integrands (OSCILLATORY_QUADRATIC(_LINEAR))
 *   run on the complex sweep, whose forward sweep follows the plan's
 *   precision mode and whose reverse sweep (sg_plan_execute_grad) is FP64
 *   whatever the mode. */
typedef struct {
    uint64_t effective_points;
    uint64_t units;
    uint64_t pair_evals;
    uint64_t macs;
    uint64_t merge_flops;
    int32_t block_threads;
    int32_t grid_blocks;
    int32_t coords_per_lane;
    int32_t max_group;
    int32_t graph;
    int32_t persistent;
    int32_t cost_scaled;
    int32_t balanced;
    int32_t fp64_complex;
    int32_t reserved;
} sg_plan_info;

sg_status sg_plan_get_info(const sg_plan *plan, sg_plan_info *info);

/* Time candidate schedules for this plan on `stream` with HIP events and
 * keep the fastest (stored in the context; later plans with the same shape
 * class reuse it): the integrand-to-wave schedule (coordinates per lane
 * 1, 2, 3, 4, 8, 16, uniform or cost-scaled, times waves per integrand
 * 1, 2, 4; and the balanced schedule with 1..4 waves per SIMD; see
 * sg_plan_info),
 * hardware dispatch versus the persistent work-queue kernel and, on a
 * non-default stream, graph replay versus direct launch.  Runs the forward
 * launch repeatedly on params_dev/out_dev (their contents are overwritten).
 * Errors: INVALID_ARGUMENT, DEVICE. */
sg_status sg_plan_autotune(sg_plan *plan, const double *params_dev, double *out_dev, void *stream);

/* Set the forward schedule and launch mode directly (the knobs
 * sg_plan_autotune chooses; see sg_plan_info): coords_per_lane in 1..64,
 * max_group in {1, 2, 4}, cost_scaled 0/1, persistent 0/1, graph 0 (direct
 * launch) or 1 (graph replay on non-default streams).  Re-packs the plan's
 * workgroups; synchronous.  Errors: INVALID_ARGUMENT, OUT_OF_MEMORY, DEVICE. */
sg_status sg_plan_set_schedule(sg_plan *plan, int32_t coords_per_lane, int32_t max_group,
                               int32_t cost_scaled, int32_t persistent, int32_t graph);

/* Balanced forward schedule: every wave of the forward launch gets about
 * the same estimated cost and the launch has at most waves_per_simd waves
 * per SIMD of the device.  A cost model of the kernel (per coordinate: node
 * pairs and weighted terms of the problem's class and precision mode; per
 * wave: the loads, the reduction across lanes and the read-out) picks the
 * coordinates per lane of each class for one common target wave cost, the
 * smallest target whose waves fit; waves form 4-wave workgroups of similar
 * cost, and the workgroups are ordered so that each compute unit receives
 * the same load under the hardware's in-order placement (workgroup i on
 * compute unit i mod the unit count while all are resident).  Uses hardware
 * dispatch (no persistent queue); graph: as for sg_plan_set_schedule.  Only
 * the speed depends on the schedule, never the values beyond the order of
 * the sweep's products.
 * Errors: INVALID_ARGUMENT (waves_per_simd outside 1..8, graph not 0/1),
 * OUT_OF_MEMORY, DEVICE. */
sg_status sg_plan_set_schedule_balanced(sg_plan *plan, int32_t waves_per_simd, int32_t graph);

/* Release a plan (NULL accepted). */
sg_status sg_plan_destroy(sg_plan *plan);

/* Literal point-by-point evaluation of (2.6)-(2.7) for one integrand: every
 * multi-index of the window is unranked on the device (chunks of 64 ranks
 * per wave), its tensor rule expanded over the points with the
 * per-coordinate node contributions staged in LDS, and
 * f(c) + sum coef(|l|) sum w (f(x) - f(c)) accumulated in double-double.
 * Cost is proportional to n_d^q (sg_counts): the call fails with
 * UNSUPPORTED when n_d^q > max_points (0 = no limit).  FP64 point values.
 * params_dev: this integrand's parameters (param_offset ignored);
 * out_dev: one float64 (device-accessible); bound_dev: NULL or one float64,
 * an a-priori rounding bound 16 * 2^-53 * (S + |f(c)|), S the sum over
 * points of |coef w| (|f(x) - f(c)| + |f(x)| |x - c|-weighted partial
 * quantity) (the terms' cancellation makes this path far less accurate than
 * the sweep at large d).  The context's workspace is reused by every call: calls on one
 * context must not overlap in time.
 * Errors: INVALID_ARGUMENT, UNSUPPORTED, OVERFLOW, OUT_OF_MEMORY, DEVICE. */
sg_status sg_integrate_points(sg_context *ctx, const sg_problem *problem, const double *params_dev,
                              double *out_dev, double *bound_dev, uint64_t max_points, void *stream);

/* Plain, plan-free path: one integrand, one launch, no graph, no batching.
 * Same arguments as one problem of a plan (param_offset is ignored: params_dev
 * points at this integrand's parameters).  out_dev/bound_dev: one float64
 * each (bound may be NULL).  Up to d = 2048 (512 for the two
 * OSCILLATORY_QUADRATIC families) one workgroup of 256 lanes sweeps every
 * coordinate; larger integrands are split over ceil(d / 256) workgroups (at
 * most 1024), one coordinate per lane and pass; each workgroup reduces its
 * chunk to a partial truncated product, and the last workgroup to finish
 * joins the partials in a fixed order (deterministic) and reads out the
 * value and bound (the associative product of Section 3, (3.9)-(3.11), split
 * by chunks).  The partials use a scratch buffer the context allocates on
 * the first split call (about 160 KiB, kept until the context is
 * destroyed); calls on one
 * context must not overlap in time.  Also takes OSCILLATORY_QUADRATIC(_LINEAR) in
 * every precision mode: the sweep of Section 3 with the complex surpluses of
 * e^{i a (x - u)^2} (FP32 node values in the FP32 modes, FP64 complex
 * products and read-out) and the bound of the real sweep (complex moduli in
 * place of absolute values). */
sg_status sg_integrate(sg_context *ctx, const sg_problem *problem, int32_t precision,
                       const double *params_dev, double *out_dev, double *bound_dev, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * computation, launches and results as sg_integrate, bit for bit, with the
 * split launches' scratch in a fixed array the library's code object
 * carries (one per GPU, kept until the process ends; its address is taken
 * once per device by sg_context_create).  Allocates nothing: no hipMalloc,
 * hipFree or allocating library routine.  The array holds 1024 partials
 * (about 160 KiB); problems never need more (the workgroup count is capped
 * at 1024, more coordinates per lane beyond), and a request that would is
 * rejected with UNSUPPORTED before launching.  Every call on one GPU shares
 * the array, so calls that overlap in time on one GPU race (their results
 * are undefined); calls in sequence on one stream are safe, and each
 * completed call leaves the array ready for the next.
 * Errors: as sg_integrate; DEVICE if the context has no array address. */
sg_status sg_integrate_noalloc(sg_context *ctx, const sg_problem *problem, int32_t precision,
                               const double *params_dev, double *out_dev, double *bound_dev, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* SGMDI_H */
