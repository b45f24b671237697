// Reverse-sweep kernels, precision 0; a plan holding gaussian problems
// launches the instantiation built with that family.
#include "sg_device.hpp"

namespace sg {

int launch_adjoint_p0(bool gauss, int nwg, const WGDesc* wgs, const ProbDev* probs, const double* pool64,
                       const float* pool32, const double* params, const double* gout, double* grad, double* ws,
                       void* stream)
{
    if (nwg <= 0) return 0;
    const dim3 grid((unsigned)nwg), block(256);
    if (gauss)
        hipLaunchKernelGGL((dev::k_adjoint<0, true>), grid, block, 0, (hipStream_t)stream, wgs, probs, pool64,
                           pool32, params, gout, grad, ws);
    else
        hipLaunchKernelGGL((dev::k_adjoint<0>), grid, block, 0, (hipStream_t)stream, wgs, probs, pool64, pool32,
                           params, gout, grad, ws);
    return (int)hipGetLastError();
}

}  // namespace sg
