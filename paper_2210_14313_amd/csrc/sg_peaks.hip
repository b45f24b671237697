// Per-operation VALU ceiling probe (include/sgpeaks.h).
//
// Each kernel runs eight independent dependency chains per lane of one
// operation class, so the latency of a chain is hidden by the other chains
// and by the other resident waves, and the class's issue rate bounds the
// kernel.  The operands are per-lane values (vector registers), so the
// compiler emits the encoding named in the header: x = fma(a, b, x) becomes
// the VOP2 v_fmac (accumulator = destination), x = fma(x, a, b) the VOP3
// v_fma.  The chains' results feed a store that never happens (the
// comparison value is a runtime argument the chains cannot reach), so every
// operation is kept.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sgpeaks.h"

namespace {

template <int OP, class T>
__device__ __forceinline__ T step(T x, T a, T b)
{
    if constexpr (OP == SGP_FMAC_F32 || OP == SGP_FMAC_F64) return __builtin_fma(a, b, x);
    else if constexpr (OP == SGP_FMA_F32 || OP == SGP_FMA_F64) return __builtin_fma(x, a, b);
    else if constexpr (OP == SGP_ADD_F32 || OP == SGP_ADD_F64) return x + a;
    else if constexpr (OP == SGP_EXP_F32) return __builtin_amdgcn_exp2f(x);
    else if constexpr (OP == SGP_SIN_F32) return __builtin_amdgcn_sinf(x);
    else if constexpr (OP == SGP_COS_F32) return __builtin_amdgcn_cosf(x);
    else if constexpr (OP == SGP_RCP_F32) return __builtin_amdgcn_rcpf(x);
    else if constexpr (OP == SGP_LOG_F32) return __builtin_amdgcn_logf(x);
    else return __builtin_amdgcn_rcp(x);   // SGP_RCP_F64
}

template <>
__device__ __forceinline__ float step<SGP_FMAC_F32, float>(float x, float a, float b)
{
    return __builtin_fmaf(a, b, x);
}
template <>
__device__ __forceinline__ float step<SGP_FMA_F32, float>(float x, float a, float b)
{
    return __builtin_fmaf(x, a, b);
}

template <int OP, class T>
__global__ void __launch_bounds__(256) k_peak(double* __restrict__ sink, int iters, T never)
{
    const T a = (T)0.999 + (T)1e-6 * (T)threadIdx.x, b = (T)1e-3 + (T)1e-7 * (T)threadIdx.x;
    T x[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) x[i] = (T)0.25 + (T)1e-6 * (T)(threadIdx.x + 64 * i);
#pragma unroll 4
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int i = 0; i < 8; ++i) x[i] = step<OP, T>(x[i], a, b);
    }
    T s = 0;
#pragma unroll
    for (int i = 0; i < 8; ++i) s += x[i];
    if (s == never) sink[blockIdx.x] = (double)s;
}

// One exponential and one VOP2 FMA per chain step, on separate chains.
__global__ void __launch_bounds__(256) k_peak_mix(double* __restrict__ sink, int iters, float never)
{
    const float a = 0.999f + 1e-6f * (float)threadIdx.x, b = 1e-3f + 1e-7f * (float)threadIdx.x;
    float x[8], y[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        x[i] = 0.25f + 1e-6f * (float)(threadIdx.x + 64 * i);
        y[i] = x[i] + 0.5f;
    }
#pragma unroll 4
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            x[i] = __builtin_amdgcn_exp2f(x[i]);
            y[i] = __builtin_fmaf(a, b, y[i]);
        }
    }
    float s = 0.0f;
#pragma unroll
    for (int i = 0; i < 8; ++i) s += x[i] + y[i];
    if (s == never) sink[blockIdx.x] = (double)s;
}

template <int OP, class T>
void launch(int blocks, int iters, double* sink, hipStream_t st)
{
    hipLaunchKernelGGL((k_peak<OP, T>), dim3(blocks), dim3(256), 0, st, sink, iters, (T)-12345.678);
}

}  // namespace

extern "C" int32_t sgp_launch(int32_t op, int32_t blocks, int32_t iters, double* sink_dev, void* stream,
                              double* ops_per_launch, double* flops_per_op)
{
    if (op < 0 || op >= SGP_NUM_OPS || blocks < 1 || iters < 1 || sink_dev == nullptr) return 1;
    hipStream_t st = (hipStream_t)stream;
    switch (op) {
    case SGP_FMAC_F32: launch<SGP_FMAC_F32, float>(blocks, iters, sink_dev, st); break;
    case SGP_FMA_F32: launch<SGP_FMA_F32, float>(blocks, iters, sink_dev, st); break;
    case SGP_ADD_F32: launch<SGP_ADD_F32, float>(blocks, iters, sink_dev, st); break;
    case SGP_FMAC_F64: launch<SGP_FMAC_F64, double>(blocks, iters, sink_dev, st); break;
    case SGP_FMA_F64: launch<SGP_FMA_F64, double>(blocks, iters, sink_dev, st); break;
    case SGP_ADD_F64: launch<SGP_ADD_F64, double>(blocks, iters, sink_dev, st); break;
    case SGP_EXP_F32: launch<SGP_EXP_F32, float>(blocks, iters, sink_dev, st); break;
    case SGP_SIN_F32: launch<SGP_SIN_F32, float>(blocks, iters, sink_dev, st); break;
    case SGP_COS_F32: launch<SGP_COS_F32, float>(blocks, iters, sink_dev, st); break;
    case SGP_RCP_F32: launch<SGP_RCP_F32, float>(blocks, iters, sink_dev, st); break;
    case SGP_LOG_F32: launch<SGP_LOG_F32, float>(blocks, iters, sink_dev, st); break;
    case SGP_RCP_F64: launch<SGP_RCP_F64, double>(blocks, iters, sink_dev, st); break;
    default:
        hipLaunchKernelGGL(k_peak_mix, dim3(blocks), dim3(256), 0, st, sink_dev, iters, -12345.678f);
        break;
    }
    if (hipGetLastError() != hipSuccess) return 5;
    const double ops = (double)blocks * 256.0 * 8.0 * (double)iters;
    const bool fma = op == SGP_FMAC_F32 || op == SGP_FMA_F32 || op == SGP_FMAC_F64 || op == SGP_FMA_F64;
    if (ops_per_launch) *ops_per_launch = op == SGP_MIX_EXP_FMAC_F32 ? 2.0 * ops : ops;
    if (flops_per_op) *flops_per_op = fma ? 2.0 : op == SGP_MIX_EXP_FMAC_F32 ? 1.5 : 1.0;
    return 0;
}

extern "C" const char* sgp_op_name(int32_t op)
{
    static const char* names[SGP_NUM_OPS] = {"v_fmac_f32", "v_fma_f32", "v_add_f32", "v_fmac_f64", "v_fma_f64",
                                             "v_add_f64", "v_exp_f32", "v_sin_f32", "v_cos_f32", "v_rcp_f32",
                                             "v_log_f32", "v_rcp_f64", "v_exp_f32+v_fmac_f32"};
    return (op >= 0 && op < SGP_NUM_OPS) ? names[op] : "";
}
