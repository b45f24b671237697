// One integrand of the dimension sweep on several workgroups (sg_one.hpp),
// precision mode 1 (FP32 values, two-sum compensated FP32 sums).
#include "sg_one.hpp"

namespace sg {
template int launch_one_inst<1>(int, int, int, int, int, const double*, double*, double*, double*, void*);
}  // namespace sg
