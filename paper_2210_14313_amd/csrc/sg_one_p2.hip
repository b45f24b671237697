// One integrand of the dimension sweep on several workgroups (sg_one.hpp),
// precision mode 2 (FP32 values, FP64 sums).
#include "sg_one.hpp"

namespace sg {
template int launch_one_inst<2>(int, int, int, int, int, const double*, double*, double*, double*, void*);
}  // namespace sg
