// Forward-sweep kernels, precision 1: one instantiation per largest
// excess budget class (K <= 4, <= 6, <= 8); a plan launches the smallest
// class covering its problems (fewer registers, more waves per SIMD); a
// plan holding gaussian problems launches the K <= 8 kernel built with the
// gaussian family (launch class kKmaxGauss).
#include "sg_device.hpp"

namespace sg {

int launch_forward_p1(int kmax, int nwg, const FwdWG* wgs, unsigned int* queue, int qgrid, const double* pool64,
                      const float* pool32, const double* params, double* out, double* bound, void* stream)
{
    if (nwg <= 0) return 0;
    const dim3 block(256), grid((unsigned)(queue ? qgrid : nwg));
    hipStream_t s = (hipStream_t)stream;
    if (kmax <= 4)
        hipLaunchKernelGGL((dev::k_forward<1, 4>), grid, block, 0, s, wgs, nwg, queue, pool64, pool32, params, out,
                           bound);
    else if (kmax <= 6)
        hipLaunchKernelGGL((dev::k_forward<1, 6>), grid, block, 0, s, wgs, nwg, queue, pool64, pool32, params, out,
                           bound);
    else if (kmax <= 8)
        hipLaunchKernelGGL((dev::k_forward<1, 8>), grid, block, 0, s, wgs, nwg, queue, pool64, pool32, params, out,
                           bound);
    else   // kKmaxGauss: a plan with gaussian problems
        hipLaunchKernelGGL((dev::k_forward<1, 8, true>), grid, block, 0, s, wgs, nwg, queue, pool64, pool32, params,
                           out, bound);
    return (int)hipGetLastError();
}

// Workgroups of the persistent forward kernel the current device holds at
// once (resident capacity), 0 on error.
int forward_capacity_p1(int kmax)
{
    const void* f = kmax <= 4   ? reinterpret_cast<const void*>(&dev::k_forward<1, 4>)
                    : kmax <= 6 ? reinterpret_cast<const void*>(&dev::k_forward<1, 6>)
                    : kmax <= 8 ? reinterpret_cast<const void*>(&dev::k_forward<1, 8>)
                                : reinterpret_cast<const void*>(&dev::k_forward<1, 8, true>);
    int per_cu = 0, dev = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, f, 256, 0) != hipSuccess) return 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    return per_cu * cus;
}

}  // namespace sg
