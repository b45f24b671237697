// Launch and occupancy query of one forward-sweep kernel instantiation
// (precision mode P, largest excess budget class KM, gaussian family G).
// Each sg_fwd_p*_*.hip unit instantiates exactly one of these, so the
// kernels compile in parallel; sg_unrank.hip dispatches to them.
#pragma once
#include "sg_device.hpp"

namespace sg {

template <int P, int KM, bool G>
int launch_forward_inst(int nwg, const FwdWG* wgs, unsigned int* queue, int qgrid, const double* pool64,
                        const float* pool32, const double* params, double* out, double* bound, void* stream)
{
    if (nwg <= 0) return 0;
    const dim3 block(256), grid((unsigned)(queue ? qgrid : nwg));
    hipLaunchKernelGGL((dev::k_forward<P, KM, G>), grid, block, 0, (hipStream_t)stream, wgs, nwg, queue, pool64,
                       pool32, params, out, bound);
    return (int)hipGetLastError();
}

// Workgroups of the persistent form the current device holds at once
// (resident capacity), 0 on error.
template <int P, int KM, bool G>
int forward_capacity_inst()
{
    int per_cu = 0, dev = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(&dev::k_forward<P, KM, G>),
                                                     256, 0) != hipSuccess)
        return 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    return per_cu * cus;
}

#define SG_FORWARD_INSTANCE(P, KM, G)                                                                            \
    template int launch_forward_inst<P, KM, G>(int, const FwdWG*, unsigned int*, int, const double*, const float*, \
                                               const double*, double*, double*, void*);                          \
    template int forward_capacity_inst<P, KM, G>();

}  // namespace sg
