// Oscillatory-quadratic sweep (complex surpluses and truncated products,
// FP64): descriptors and launchers shared by the kernel file and the API.
#pragma once

#include <cstdint>

namespace sg {

// One oscillatory-quadratic integrand of a plan.
struct OscqDesc {
    int64_t off64;          // its (rule, K) record table in the plan's FP64 pool
    int64_t param_offset;   // its parameters w, a[d], u[d] in the caller's array
    int32_t d, K, rule;
    int32_t out_index;      // its slot in out / bound
    int64_t ws_off;         // reverse sweep: its d * 2K doubles in the workspace
};

// One integrand (the plan-free path) on G workgroups: pool64 holds the
// (rule, K) record table, or is NULL for the tables compiled into the
// library; out and bound (NULL: none) one double each;
// scratch (G > 1): kOscqScratchHead + G * kOscqWords doubles whose first
// 32-bit word, the arrival counter, is zero, and is left zero.
constexpr int kOscqScratchHead = 32;
constexpr int kOscqWords = 2 * 8 + 4;
int launch_oscq(int d, int K, int rule, int G, const double* pool64, const double* params, double* out,
                double* bound, double* scratch, void* stream);
// n integrands of a plan, one workgroup each; out and bound (NULL: none)
// indexed by out_index.
int launch_oscq_batch(int n, const OscqDesc* descs, const double* pool64, const double* params, double* out,
                      double* bound, void* stream);
// Reverse sweep of n integrands of a plan, one workgroup each: grad (the
// parameters' layout) receives gout[out_index] times the gradient of each
// integrand's value; ws: the plan's workspace (OscqDesc::ws_off).
int launch_oscq_grad(int n, const OscqDesc* descs, const double* pool64, const double* params, const double* gout,
                     double* grad, double* ws, void* stream);

}  // namespace sg
