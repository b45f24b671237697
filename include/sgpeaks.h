/*
 * sgpeaks.h -- C ABI of the per-operation VALU ceiling probe for MI355X
 * (gfx950), libsgpeaks.so.
 *
 * The roofline of the dimension sweep is a serial-issue model over the
 * operation classes the method must execute: T_min = sum_op n_op / peak_op,
 * with n_op the algorithmic counts per (integrand, coordinate) unit (node
 * evaluations of the 1-D rules of Section 2.2, within-rule multiply-adds of
 * the hierarchical sums of (2.9), truncated-polynomial products of the
 * dimension iteration (3.9)-(3.11)) and peak_op the rate of that class on
 * the device.  This library measures the rates on the device instead of
 * taking them from a data sheet: each probe kernel issues one operation
 * class in eight independent dependency chains per lane, over a grid that
 * keeps eight waves resident on every SIMD, so the issue rate of the class
 * is what limits it.  The caller times the launch (e.g. with HIP events on
 * the same stream) and divides.
 *
 * Packed FP32 instructions are not used (the library is built without
 * them).  Multiply-adds are probed in both encodings the compiler emits,
 * VOP2 (v_fmac_*: the accumulator is the destination, the other operands
 * vector registers) and VOP3 (v_fma_*: three free operands), because their
 * issue rates differ on this device; the ceiling of a class is the best
 * rate among its encodings.
 */
#ifndef SGPEAKS_H
#define SGPEAKS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SGP_FMAC_F32 = 0, /* v_fmac_f32 (VOP2, accumulator = destination; 2 flops) */
    SGP_FMA_F32 = 1,  /* v_fma_f32  (VOP3, three vector operands; 2 flops) */
    SGP_ADD_F32 = 2,  /* v_add_f32  (VOP2; 1 flop) */
    SGP_FMAC_F64 = 3, /* v_fmac_f64 (VOP2; 2 flops) */
    SGP_FMA_F64 = 4,  /* v_fma_f64  (VOP3; 2 flops) */
    SGP_ADD_F64 = 5,  /* v_add_f64  (1 flop) */
    SGP_EXP_F32 = 6,  /* v_exp_f32  (1 op) */
    SGP_SIN_F32 = 7,  /* v_sin_f32  (1 op) */
    SGP_COS_F32 = 8,  /* v_cos_f32  (1 op) */
    SGP_RCP_F32 = 9,  /* v_rcp_f32  (1 op) */
    SGP_LOG_F32 = 10, /* v_log_f32  (1 op) */
    SGP_RCP_F64 = 11, /* v_rcp_f64  (1 op) */
    SGP_MIX_EXP_FMAC_F32 = 12, /* per chain step one v_exp_f32 and one v_fmac_f32 on
                                  independent chains (2 ops, 3 "flops": 1 + 2);
                                  shows whether the two classes share issue */
    SGP_NUM_OPS = 13
} sgp_op;

/* Launch one probe kernel of operation class `op` on `stream` (a
 * hipStream_t as void*, NULL = default stream): `blocks` workgroups of 256
 * threads, each thread running `iters` steps of 8 independent chains.
 * sink_dev: device buffer of at least `blocks` doubles (written only under a
 * data-dependent condition that does not hold, so the chains are kept).
 * On return *ops_per_launch = blocks * 256 * 8 * iters operations issued
 * (for SGP_MIX_EXP_FMAC_F32, twice that: one of each class per step) and
 * *flops_per_op = 2 for FMAs, 1 otherwise (1.5 for the mix).  Either output
 * pointer may be NULL.  Asynchronous.
 * Returns 0 on success, 1 for an invalid argument (unknown op, blocks < 1,
 * iters < 1, NULL sink), 5 if the launch failed. */
int32_t sgp_launch(int32_t op, int32_t blocks, int32_t iters, double *sink_dev, void *stream,
                   double *ops_per_launch, double *flops_per_op);

/* Static name of an operation class ("v_fmac_f32", ...), or "" if unknown. */
const char *sgp_op_name(int32_t op);

#ifdef __cplusplus
}
#endif

#endif /* SGPEAKS_H */
