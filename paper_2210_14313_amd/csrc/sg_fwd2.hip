// Forward-sweep kernels, precision 2 (FP32 node values, FP64 sums): one instantiation per largest
// excess budget class (K <= 4, <= 6, <= 8); a plan launches the smallest
// class covering its problems (fewer registers, more waves per SIMD).
#include "sg_device.hpp"

namespace sg {

int launch_forward_p2(int kmax, int nwg, const FwdWG* wgs, const double* pool64,
                       const float* pool32, const double* params, double* out, double* bound, void* stream)
{
    if (nwg <= 0) return 0;
    const dim3 grid((unsigned)nwg), block(256);
    hipStream_t s = (hipStream_t)stream;
    if (kmax <= 4)
        hipLaunchKernelGGL((dev::k_forward<2, 4>), grid, block, 0, s, wgs, pool64, pool32, params, out, bound);
    else if (kmax <= 6)
        hipLaunchKernelGGL((dev::k_forward<2, 6>), grid, block, 0, s, wgs, pool64, pool32, params, out, bound);
    else
        hipLaunchKernelGGL((dev::k_forward<2, 8>), grid, block, 0, s, wgs, pool64, pool32, params, out, bound);
    return (int)hipGetLastError();
}

}  // namespace sg
