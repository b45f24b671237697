// Oscillatory-quadratic sweep (complex surpluses and truncated products):
// descriptors and launchers shared by the kernel files and the API.
#pragma once

#include <cstdint>

namespace sg {

// One oscillatory-quadratic integrand of a plan (lin: with the linear term,
// parameters w, a[d], u[d], c[d]; else w, a[d], u[d]).
struct OscqDesc {
    int64_t off64;          // its (rule, K) record table in the plan's FP64 pool
    int64_t off32;          // and in its FP32 pool (hi + lo weights)
    int64_t param_offset;   // its parameters w, a[d], u[d] in the caller's array
    int32_t d, K, rule;
    int32_t out_index;      // its slot in out / bound
    int64_t ws_off;         // reverse sweep: its d * 2K doubles in the workspace
    int32_t lin;
    int32_t reserved;
};

// One integrand (the plan-free path) on G workgroups in precision mode
// `precision` (SG_PREC_*), lin as in OscqDesc: pool64 / pool32 hold the (rule, K) record tables,
// or pool64 is NULL for the tables compiled into the library; out and bound
// (NULL: none) one double each; scratch (G > 1): kOscqScratchHead +
// G * kOscqWords doubles whose first 32-bit word, the arrival counter, is
// zero, and is left zero.
constexpr int kOscqScratchHead = 32;
constexpr int kOscqWords = 2 * 8 + 4;
int launch_oscq(int precision, int d, int K, int rule, int G, int lin, const double* pool64, const float* pool32,
                const double* params, double* out, double* bound, double* scratch, void* stream);
// n integrands of a plan, one workgroup each; out and bound (NULL: none)
// indexed by out_index.
int launch_oscq_batch(int precision, int n, const OscqDesc* descs, const double* pool64, const float* pool32,
                      const double* params, double* out, double* bound, void* stream);
// The same for one precision mode (PREC = SG_PREC_*).
template <int PREC>
int launch_oscq_prec(int d, int K, int rule, int G, int lin, const double* pool64, const float* pool32,
                     const double* params, double* out, double* bound, double* scratch, void* stream);
template <int PREC>
int launch_oscq_batch_prec(int n, const OscqDesc* descs, const double* pool64, const float* pool32,
                           const double* params, double* out, double* bound, void* stream);
// Reverse sweep of n integrands of a plan, one workgroup each: grad (the
// parameters' layout) receives gout[out_index] times the gradient of each
// integrand's value; ws: the plan's workspace (OscqDesc::ws_off).
int launch_oscq_grad(int n, const OscqDesc* descs, const double* pool64, const double* params, const double* gout,
                     double* grad, double* ws, void* stream);

}  // namespace sg
